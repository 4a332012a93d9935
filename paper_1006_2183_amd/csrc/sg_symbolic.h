// Symbolic-phase kernels: output vector lists, AUX lookup, flops per output
// vector, tier binning, window split points and device-wide scans.
#pragma once

#include "sg_device.h"

namespace sg {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- exclusive scan of int64 (out[n] = total), three passes -----------------
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int64_t *in, int64_t n, int64_t *part) {
  __shared__ int64_t scratch[kMaxWaves + 1];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t x = base + (int64_t)threadIdx.x * kScanItems + i;
    if (x < n) s += in[x];
  }
  int64_t tot = block_sum(s, scratch);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_partials(int64_t *part, int64_t nb) {
  __shared__ int64_t scratch[kMaxWaves + 1];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {
    int64_t x = b0 + threadIdx.x;
    int64_t v = x < nb ? part[x] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, scratch, &tot);
    if (x < nb) part[x] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

// Small scans in one launch: 1024 threads, each sums its run of consecutive
// elements, one block-wide scan of the run totals, then each thread writes
// its run (n <= kSmallScan).
constexpr int64_t kSmallScan = 16384;
__global__ void __launch_bounds__(1024) k_scan_small(const int64_t *in, int64_t n, int64_t *out) {
  __shared__ int64_t scratch[kMaxWaves + 1];
  const int64_t per = (n + blockDim.x - 1) / blockDim.x;
  const int64_t a = (int64_t)threadIdx.x * per < n ? (int64_t)threadIdx.x * per : n;
  const int64_t b = a + per < n ? a + per : n;
  int64_t s = 0;
  for (int64_t i = a; i < b; ++i) s += in[i];
  int64_t tot;
  int64_t run = block_excl_scan(s, scratch, &tot);
  for (int64_t i = a; i < b; ++i) {
    const int64_t x = in[i];
    out[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) out[n] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(const int64_t *in, int64_t n, const int64_t *part,
                                                           int64_t nb, int64_t *out) {
  __shared__ int64_t scratch[kMaxWaves + 1];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(s, scratch, &tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = part[nb];
}

// ---- AUX index of a doubly compressed matrix (Section 2.3) -----------------
__global__ void k_build_aux(const int32_t *vid, int64_t nvec, int64_t chunk, int64_t nchunks, int32_t *aux) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > nchunks) return;
  if (c == nchunks) {
    aux[c] = (int32_t)nvec;
    return;
  }
  int64_t key = c * chunk;
  int64_t lo = 0, hi = nvec;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (vid[mid] < key) lo = mid + 1; else hi = mid;
  }
  aux[c] = (int32_t)lo;
}

// ---- output vectors when every group holds a single product ---------------
// Output vector v is stored vector t of product p's S, v = vbase[p] + t.
__global__ void k_ov_simple(const ProdDev *prods, const int64_t *vbase, int32_t nprod, int64_t nov,
                            int32_t *ov_id, int32_t *ov_group, int64_t *ov_seg, int32_t *seg_prod,
                            int32_t *seg_svec, int64_t *counters) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counters[kCtNov] = nov;
    counters[kCtNseg] = nov;
    ov_seg[0] = 0;
  }
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nov; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nprod - 1;
    while (lo < hi) {  // last p with vbase[p] <= v
      int32_t mid = (lo + hi + 1) >> 1;
      if (vbase[mid] <= v) lo = mid; else hi = mid - 1;
    }
    const ProdDev &d = prods[lo];
    int64_t t = v - vbase[lo];
    ov_id[v] = d.s_vid ? d.s_vid[t] : (int32_t)t;
    ov_group[v] = d.group;
    ov_seg[v] = v;
    seg_prod[v] = lo;
    seg_svec[v] = (int32_t)t;
    if (v == nov - 1) ov_seg[nov] = nov;
  }
}

// ---- output vectors of groups with several products (stage merge) ---------
// A dense count per output major id of each group (dbase[g] + j), then two
// scans give the output vector numbering and the segment offsets.
__global__ void k_dense_count(const ProdDev *prods, const int64_t *vbase, int32_t nprod, int64_t nvec_all,
                              const int64_t *dbase, int64_t *dcnt) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nvec_all; x += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nprod - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (vbase[mid] <= x) lo = mid; else hi = mid - 1;
    }
    const ProdDev &d = prods[lo];
    int64_t t = x - vbase[lo];
    int64_t j = d.s_vid ? d.s_vid[t] : t;
    if (d.s_ptr[t + 1] > d.s_ptr[t])
      atomicAdd((unsigned long long *)&dcnt[dbase[d.group] + j], 1ull);
  }
}

__global__ void k_nonzero_flag(const int64_t *in, int64_t n, int64_t *out) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    out[x] = in[x] > 0 ? 1 : 0;
}

__global__ void k_dense_emit(const int64_t *dcnt, const int64_t *vpos, const int64_t *spos, int64_t ndense,
                             const int64_t *dbase, int32_t ngroup, int32_t *ov_id, int32_t *ov_group,
                             int64_t *ov_seg, int64_t *counters) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < ndense; x += (int64_t)gridDim.x * blockDim.x) {
    if (x == ndense - 1) {
      counters[kCtNov] = vpos[ndense];
      counters[kCtNseg] = spos[ndense];
      ov_seg[vpos[ndense]] = spos[ndense];
    }
    if (dcnt[x] == 0) continue;
    int32_t lo = 0, hi = ngroup - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (dbase[mid] <= x) lo = mid; else hi = mid - 1;
    }
    int64_t v = vpos[x];
    ov_id[v] = (int32_t)(x - dbase[lo]);
    ov_group[v] = lo;
    ov_seg[v] = spos[x];
  }
}

__global__ void k_dense_segs(const ProdDev *prods, const int64_t *vbase, int32_t nprod, int64_t nvec_all,
                             const int64_t *dbase, const int64_t *spos, int64_t *dfill, int32_t *seg_prod,
                             int32_t *seg_svec) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nvec_all; x += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nprod - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (vbase[mid] <= x) lo = mid; else hi = mid - 1;
    }
    const ProdDev &d = prods[lo];
    int64_t t = x - vbase[lo];
    if (d.s_ptr[t + 1] == d.s_ptr[t]) continue;
    int64_t j = d.s_vid ? d.s_vid[t] : t;
    int64_t dx = dbase[d.group] + j;
    int64_t slot = spos[dx] + (int64_t)atomicAdd((unsigned long long *)&dfill[dx], 1ull);
    seg_prod[slot] = lo;
    seg_svec[slot] = (int32_t)t;
  }
}

// Order the segments of each output vector by product (deterministic order).
__global__ void k_sort_segs(const int64_t *ov_seg, const int64_t *counters, int32_t *seg_prod, int32_t *seg_svec) {
  int64_t nov = counters[kCtNov];
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nov; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = ov_seg[v], b = ov_seg[v + 1];
    for (int64_t i = a + 1; i < b; ++i) {
      int32_t p = seg_prod[i], t = seg_svec[i];
      int64_t j = i - 1;
      while (j >= a && seg_prod[j] > p) {
        seg_prod[j + 1] = seg_prod[j];
        seg_svec[j + 1] = seg_svec[j];
        --j;
      }
      seg_prod[j + 1] = p;
      seg_svec[j + 1] = t;
    }
  }
}

// Group ranges of output vectors (ov ids are ordered by group).
__global__ void k_group_ranges(const int32_t *ov_group, const int64_t *counters, GroupDev *groups, int32_t ngroup) {
  int64_t nov = counters[kCtNov];
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroup) return;
  int64_t lo = 0, hi = nov;  // first v with ov_group[v] >= g
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (ov_group[mid] < g) lo = mid + 1; else hi = mid;
  }
  int64_t b = lo;
  hi = nov;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (ov_group[mid] <= g) lo = mid + 1; else hi = mid;
  }
  groups[g].ov_begin = b;
  groups[g].ov_end = lo;
}

// ---- flops per output vector (one wavefront per vector) --------------------
// flops_j = sum over stored (k, s) of S(:, j) of nnz(G(:, k)); a k with an
// empty G vector contributes nothing (the Isect observation, Section 2.4).
// For a doubly compressed G the resolved vector is kept per S entry.
// ---- tier binning -----------------------------------------------------------
// Wave-aggregated append of this lane's vector to list `which` if `take`.
__device__ __forceinline__ void append(bool take, int32_t v, int32_t *list, int64_t *counter) {
  uint64_t m = __ballot(take);
  if (m == 0) return;
  int leader = __ffsll((unsigned long long)m) - 1;
  int64_t base = 0;
  if (lane() == leader) base = (int64_t)atomicAdd((unsigned long long *)counter, (unsigned long long)__popcll(m));
  base = __shfl(base, leader, kWave);
  uint64_t below = m & ((1ull << lane()) - 1ull);
  if (take) list[base + __popcll(below)] = v;
}

struct BinParams {
  int32_t tiny_max;
  int32_t mid_cap;
  int32_t force;
  int32_t small_max;  // mid-tier vectors up to this many products go to the small list (0: none)
};

// Products of a small-list vector at most (sixteen per lane of a wavefront),
// and the largest id range it may have (its ids are packed with a 10-bit slot
// into 32-bit sort keys, and the all-ones key is the padding).
constexpr int kSmallPerLane = 16;
constexpr int kSmallMaxFlops = kSmallPerLane * kWave;
constexpr int64_t kSmallMaxMinor = ((int64_t)1 << 22) - 1;
// Output vectors (upper bound) from which a plan uses the small list.
constexpr int64_t kSmallMinVectors = 8192;

// G vector of stored S entry e (-1: absent); a doubly compressed G is
// resolved through AUX and the result kept in d.gres for the numeric kernels.
__device__ __forceinline__ int32_t resolve_entry(const ProdDev &d, int64_t e, int32_t k) {
  if (d.g_vid) {
    const int32_t gt = aux_find(d, k);
    gstore(d.gres + e, gt);
    return gt;
  }
  return (k >= 0 && k < d.g_nvec) ? k : -1;
}

// Multiplications of the stored S entries e0 + l, e0 + l + stride, ... < e1
// (stride 1 for one lane walking a short vector, 64 for a wavefront), four
// entries in flight at a time.
__device__ __forceinline__ int64_t entries_flops(const ProdDev &d, int64_t e0, int64_t e1, int64_t stride) {
  int64_t f = 0;
  for (int64_t e = e0; e < e1; e += 4 * stride) {
    int32_t k[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = e + j * stride < e1 ? gload(d.s_idx + e + j * stride) : -1;
    int32_t gt[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) gt[j] = e + j * stride < e1 ? resolve_entry(d, e + j * stride, k[j]) : -1;
    int64_t a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = gt[j] >= 0 ? gload(d.g_ptr + gt[j]) : 0;
      b[j] = gt[j] >= 0 ? gload(d.g_ptr + gt[j] + 1) : 0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) f += b[j] - a[j];
  }
  return f;
}

// Flops per output vector, the group totals (flops, bound, largest vector)
// and the tier of every vector (appended to the tiny, mid and heavy lists,
// with per-tier flops and streamed entries). A wavefront takes 64
// consecutive output vectors, one per lane: vectors with one segment of the
// chunk's common product and at most kSerial streamed entries are summed by
// their own lane; the others by the whole wavefront, one at a time (over
// the entries of each segment, or one segment per lane when there are
// kLaneSegs segments or more and they are short).
//
// Tiers: no multiplication, none; else forced tier if any (a forced mid
// vector that does not fit goes heavy); else tiny up to tiny_max flops; mid
// when the size bound (flops capped by the id range) fits the mid
// accumulator and the id range spans several split buckets (with one bucket
// the heavy tier's single dense window is the better accumulator); else heavy.
__global__ void k_flops_bin(Plan P, BinParams bp, int64_t *gstat, int64_t *counters, int32_t *tiny, int32_t *mid,
                            int32_t *heavy, int32_t *small) {
  constexpr int kSerial = 32;
  constexpr int kLaneSegs = 8;  // segments from which a vector's segments go one per lane
  constexpr int kBatch = 8;     // chunks whose list appends share one atomic per tier
  const int l = lane();
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t nov = counters[kCtNov];
  int64_t tf[3] = {0, 0, 0}, ts[3] = {0, 0, 0};
  // group totals of the current group, flushed when the group changes
  int32_t cur_g = -1;
  int64_t acc_f = 0, acc_ub = 0, acc_max = 0;
  auto flush_group = [&]() {
    if (cur_g < 0) return;
    const int64_t sf = wave_sum64(acc_f), su = wave_sum64(acc_ub), mx = wave_max64(acc_max);
    if (l == 0) {
      atomicAdd((unsigned long long *)&gstat[cur_g * kStCount + kStFlops], (unsigned long long)sf);
      atomicAdd((unsigned long long *)&gstat[cur_g * kStCount + kStUb], (unsigned long long)su);
      atomicMax((unsigned long long *)&gstat[cur_g * kStCount + kStMaxFlops], (unsigned long long)mx);
    }
    acc_f = acc_ub = acc_max = 0;
  };
  // chunks per batch: one while the chunks do not outnumber the wavefronts.
  // With r >= 2 wavefronts per chunk, each chunk is shared by r of them:
  // sub-wave 0 takes the vectors its lanes sum alone, and the vectors summed
  // by the whole wavefront are dealt round robin to the r sub-waves (R-MAT's
  // first rows put dozens of such vectors in one chunk); every sub-wave bins
  // the vectors it summed.
  const int64_t nchunks = (nov + kWave - 1) / kWave;
  const int64_t r = nchunks >= nwaves ? 1 : nwaves / (nchunks > 0 ? nchunks : 1);
  const int64_t sub = wave % r, wv = wave / r, nwv = nwaves / r;
  const int64_t nbq = nchunks / nwv;
  const int nb = nbq < 1 ? 1 : (nbq > kBatch ? kBatch : (int)nbq);
  for (int64_t c0 = wv * nb; c0 < nchunks; c0 += nwv * nb) {
    int8_t tier_of[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int64_t v0 = (c0 + i) * kWave;
      tier_of[i] = -1;
      if (i >= nb || v0 >= nov) continue;  // uniform
      const int64_t v = v0 + l;
      const bool valid = v < nov;
      int32_t p = -1, t = 0;
      if (valid) {
        const int64_t s0 = gload(P.ov_seg + v);
        if (gload(P.ov_seg + v + 1) - s0 == 1) {
          p = gload(P.seg_prod + s0);
          t = gload(P.seg_svec + s0);
        }
      }
      const uint64_t hasp = __ballot(p >= 0);
      int64_t f = 0, sent = 0;
      bool done = false;
      if (hasp) {
        const int32_t p0 = __builtin_amdgcn_readlane(p, __ffsll((unsigned long long)hasp) - 1);
        const ProdDev d = uload(P.prods + p0);
        if (p == p0) {
          const int64_t e0 = gload(d.s_ptr + t), e1 = gload(d.s_ptr + t + 1);
          if (e1 - e0 <= kSerial) {
            if (sub == 0) f = entries_flops(d, e0, e1, 1);
            sent = e1 - e0;
            done = true;
          }
        }
      }
      uint64_t coop = __ballot(valid && !done);
      bool own = valid && done && sub == 0;  // this sub-wave bins the lane's vector
      int64_t q = 0;
      while (coop) {
        const int x = __ffsll((unsigned long long)coop) - 1;
        coop &= coop - 1ull;
        if (q++ % r != sub) continue;  // uniform: another sub-wave sums vector x
        if (l == x) own = true;
        const int64_t vx = v0 + x;
        int64_t fx = 0, sx = 0;
        const int64_t s0x = uload(P.ov_seg + vx), s1 = uload(P.ov_seg + vx + 1);
        // segments one after another, each one's entries across the lanes
        auto by_segment = [&](int64_t sa, int64_t sz) {
          for (int64_t s = sa; s < sz; ++s) {
            const ProdDev d = uload(P.prods + uload(P.seg_prod + s));
            const int32_t tt = uload(P.seg_svec + s);
            const int64_t e0 = uload(d.s_ptr + tt), e1 = uload(d.s_ptr + tt + 1);
            fx += entries_flops(d, e0 + l, e1, kWave);
            sx += e1 - e0;
          }
        };
        if (s1 - s0x >= kLaneSegs) {
          // many segments (the stage products of a SUMMA share): 64 at a
          // time, one per lane, so their descriptor chains run side by side;
          // a segment of at most four entries is then summed by its lane,
          // a longer one (a k-way merge of partials) has its entries spread
          // across the lanes
          int64_t lane_s = 0;
          for (int64_t sb = s0x; sb < s1; sb += kWave) {
            const int64_t s = sb + l;
            int64_t e0 = 0, e1 = 0;
            const ProdDev *dl = nullptr;
            if (s < s1) {
              dl = P.prods + gload(P.seg_prod + s);
              const int32_t tt = gload(P.seg_svec + s);
              const int64_t *sp = dl->s_ptr;
              e0 = gload(sp + tt);
              e1 = gload(sp + tt + 1);
            }
            const bool brief = e1 - e0 <= 4;
            if (s < s1 && brief) {
              fx += entries_flops(*dl, e0, e1, 1);
              lane_s += e1 - e0;
            }
            uint64_t longer = __ballot(s < s1 && !brief);
            while (longer) {
              const int x = __ffsll((unsigned long long)longer) - 1;
              longer &= longer - 1ull;
              by_segment(sb + x, sb + x + 1);
            }
          }
          sx += wave_sum64(lane_s);
        } else {
          by_segment(s0x, s1);
        }
        fx = wave_sum64(fx);
        if (l == x) {
          f = fx;
          sent = sx;
        }
      }
      int32_t g = -1;
      int64_t minor = 0;
      int tier = -1;
      if (own) {
        gstore(P.ov_flops + v, f);
        g = gload(P.ov_group + v);
        const GroupDev &G = P.groups[g];
        minor = gload(&G.minor);
        const int32_t mid_ok_cap = gload(&G.mid_ok);
        const int32_t nsplit = gload(&G.nsplit);
        const int64_t ub = f < minor ? f : minor;
        const bool mid_fit = mid_ok_cap > 0 && ub <= (int64_t)mid_ok_cap && ub <= (int64_t)bp.mid_cap;
        if (f == 0) tier = -1;
        else if (bp.force == 2) tier = 2;
        else if (bp.force == 1) tier = mid_fit ? 1 : 2;
        else if (bp.force == 3 && f <= kSmallMaxFlops && minor <= kSmallMaxMinor) tier = 3;
        else if (f <= bp.tiny_max) tier = 0;
        else if (f <= bp.small_max && minor <= kSmallMaxMinor) tier = 3;
        else if (mid_fit && nsplit > 1) tier = 1;
        else tier = 2;
      }
      tier_of[i] = (int8_t)tier;
      if (tier >= 0) {  // the small list counts as the mid tier in the totals
        tf[tier == 3 ? 1 : tier] += f;
        ts[tier == 3 ? 1 : tier] += sent;
      }
      // group totals: registers while the chunk stays in the current group
      const int64_t ub = f < minor ? f : minor;
      uint64_t pend = __ballot(own);
      while (pend) {
        const int32_t gx = __builtin_amdgcn_readlane(g, __ffsll((unsigned long long)pend) - 1);
        const bool mine = own && g == gx;
        pend &= ~__ballot(mine);
        if (gx != cur_g) {
          flush_group();
          cur_g = gx;
        }
        if (mine) {
          acc_f += f;
          acc_ub += ub;
          acc_max = f > acc_max ? f : acc_max;
        }
      }
    }
    // list appends of the kBatch chunks: one atomic per list
    for (int x = 0; x < 4; ++x) {
      int32_t *list = x == 0 ? tiny : (x == 1 ? mid : (x == 2 ? heavy : small));
      uint64_t m[kBatch];
      int total = 0;
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        m[i] = __ballot(tier_of[i] == x);
        total += __popcll(m[i]);
      }
      if (total == 0) continue;
      int64_t base = 0;
      if (l == 0)
        base = (int64_t)atomicAdd((unsigned long long *)&counters[x == 3 ? kCtSmall : kCtTiny + x],
                                  (unsigned long long)total);
      base = __shfl(base, 0, kWave);
      const uint64_t below = (1ull << l) - 1ull;
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        if (tier_of[i] == x) list[base + __popcll(m[i] & below)] = (int32_t)((c0 + i) * kWave + l);
        base += __popcll(m[i]);
      }
    }
  }
  flush_group();
  for (int x = 0; x < 3; ++x) {
    const int64_t a = wave_sum64(tf[x]);
    const int64_t b = wave_sum64(ts[x]);
    if (l == 0 && (a | b)) {
      atomicAdd((unsigned long long *)&counters[kCtTierFlops + x], (unsigned long long)a);
      atomicAdd((unsigned long long *)&counters[kCtTierSent + x], (unsigned long long)b);
    }
  }
}

// Output entries per tier (the small list counts as the mid tier).
__global__ void k_tier_nnz(Plan P, int64_t *counters) {
  const int64_t n[4] = {counters[kCtTiny], counters[kCtMid], counters[kCtHeavy], counters[kCtSmall]};
  const int32_t *lists[4] = {P.tiny_list, P.mid_list, P.heavy_list, P.small_list};
  for (int x = 0; x < 4; ++x) {
    int64_t acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n[x]; i += (int64_t)gridDim.x * blockDim.x)
      acc += P.ov_cnt[lists[x][i]];
    acc = wave_sum64(acc);
    const int t = x == 3 ? 1 : x;
    if (lane() == 0 && acc) atomicAdd((unsigned long long *)&counters[kCtTierNnz + t], (unsigned long long)acc);
  }
}

// Window split points of every G vector: wsplit[t * (nsplit + 1) + c] is
// the offset inside G(:, t) of the first id >= c * sw.
// Split points of every G vector at the bucket boundaries (only the heavy
// windows read them: without heavy vectors, which binning has counted by
// now, the launch does nothing).
__global__ void k_wsplit(const int64_t *g_ptr, const int32_t *g_idx, int64_t g_nvec, int32_t nsplit, int32_t sw,
                         int32_t *wsplit, const int64_t *counters) {
  if (counters[kCtHeavy] == 0) return;
  int64_t n = g_nvec * (nsplit + 1);
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = x / (nsplit + 1);
    int64_t c = x - t * (nsplit + 1);
    int64_t a = g_ptr[t], b = g_ptr[t + 1];
    int64_t lo = a, hi = b;
    int64_t key = c * (int64_t)sw;
    while (lo < hi) {
      int64_t mid = lo + ((hi - lo) >> 1);
      if (g_idx[mid] < key) lo = mid + 1; else hi = mid;
    }
    wsplit[x] = (int32_t)(lo - a);
  }
}

// Heavy-tier windows of one vector inside buckets [bs, be) (one XCD range)
// from its bucket counts. Mode 0: one window per non-empty bucket. Mode 1:
// consecutive buckets are merged while the window's LDS (the words of its
// span plus its values, in value slots) fits rank_cap, its span rank_wb
// buckets and its entries kRankMaxEntries; empty buckets between windows are
// skipped. One bucket (sw ids, at most sw entries) always fits, so each
// window takes at least one. `emit` receives (b0, b1, entries of the vector
// before b0).
constexpr int64_t kRankMaxEntries = 65504;
template <class F>
__device__ __forceinline__ int64_t plan_windows(const GroupDev &G, const int32_t *bc, int32_t bs, int32_t be,
                                                int64_t before, F emit) {
  int64_t nwin = 0;
  int32_t b = bs;
  while (b < be) {
    if (bc[b] == 0) {
      ++b;
      continue;
    }
    const int32_t b0 = b;
    int64_t sum = 0;
    if (G.mode == 0) {
      sum = bc[b];
      ++b;
    } else {
      while (b < be && (b - b0) < G.rank_wb && sum + bc[b] <= kRankMaxEntries &&
             (int64_t)(b - b0 + 1) * G.rank_wcost + sum + bc[b] <= G.rank_cap) {
        sum += bc[b];
        ++b;
      }
    }
    emit(b0, b, before);
    before += sum;
    ++nwin;
  }
  return nwin;
}

// Range r of a group covers buckets [r * bpr, min((r + 1) * bpr, nsplit)).
__device__ __forceinline__ void range_buckets(const GroupDev &G, int r, int32_t &bs, int32_t &be) {
  const int64_t s0 = (int64_t)r * G.bpr, e0 = s0 + G.bpr;
  bs = (int32_t)(s0 < G.nsplit ? s0 : G.nsplit);
  be = (int32_t)(e0 < G.nsplit ? e0 : G.nsplit);
}

// Windows per (range, heavy vector), laid out range-major: out[r * cap + q].
__global__ void k_plan_count(Plan P, int64_t cap, int64_t *nwin_out) {
  const int64_t nh = P.counters[kCtHeavy];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < cap; q += (int64_t)gridDim.x * blockDim.x) {
    if (q >= nh) {
      for (int r = 0; r < P.nrange; ++r) nwin_out[r * cap + q] = 0;
      continue;
    }
    const GroupDev &G = P.groups[P.ov_group[P.heavy_list[q]]];
    const int32_t *bc = P.bcnt + q * (int64_t)P.nbmax;
    for (int r = 0; r < P.nrange; ++r) {
      int32_t bs, be;
      range_buckets(G, r, bs, be);
      nwin_out[r * cap + q] = plan_windows(G, bc, bs, be, 0, [](int32_t, int32_t, int64_t) {});
    }
  }
}

__global__ void k_plan_fill(Plan P, const int64_t *ibase, int64_t cap, ItemDev *items, int64_t *counters,
                            const int64_t *rbase, const int32_t *vsent) {
  const int64_t nh = counters[kCtHeavy];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nh; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = P.heavy_list[q];
    const int32_t g = P.ov_group[v];
    const GroupDev &G = P.groups[g];
    const int64_t base = P.ov_off[v] - G.nnz_base;
    const int32_t *bc = P.bcnt + q * (int64_t)P.nbmax;
    const int32_t ns = vsent ? vsent[q] : 0;
    const int64_t rb = rbase ? rbase[q] : -1;
    int64_t before = 0, j = 0;
    for (int r = 0; r < P.nrange; ++r) {
      int32_t bs, be;
      range_buckets(G, r, bs, be);
      int64_t i = ibase[r * cap + q];
      plan_windows(G, bc, bs, be, before, [&](int32_t b0, int32_t b1, int64_t bef) {
        ItemDev it;
        it.v = v;
        it.g = g;
        it.b0 = b0;
        it.b1 = b1;
        it.pos = base + bef;
        it.q = (int32_t)q;
        it.nrec = ns;
        const int64_t r0 = rb + j * ns;
        it.rbase = (G.mode == 1 && ns >= 0 && rb >= 0 && r0 + ns <= P.rec_cap) ? r0 : -1;
        items[i] = it;
        ++i;
        ++j;
      });
      for (int32_t b = bs; b < be; ++b) before += bc[b];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) counters[kCtItems] = ibase[(int64_t)P.nrange * cap];
}

// Entry records of the heavy windows: per heavy vector q the stored S
// entries it streams (vsent, -1 for a vector of several segments, which
// keeps the plain walk) and the records it needs, windows x entries (rcnt,
// scanned into the record offsets).
__global__ void k_rec_count(Plan P, const int64_t *nwin, int64_t cap, int32_t *vsent, int64_t *rcnt) {
  const int64_t nh = P.counters[kCtHeavy];
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < cap; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t rc = 0;
    if (q < nh) {
      // one record per streamed entry of every segment, per window
      const int32_t v = P.heavy_list[q];
      int64_t ns = 0;
      for (int64_t s = P.ov_seg[v]; s < P.ov_seg[v + 1]; ++s) {
        const ProdDev &d = P.prods[P.seg_prod[s]];
        const int32_t t = P.seg_svec[s];
        ns += d.s_ptr[t + 1] - d.s_ptr[t];
      }
      int64_t w = 0;
      for (int r = 0; r < P.nrange; ++r) w += nwin[r * cap + q];
      vsent[q] = ns <= INT32_MAX ? (int32_t)ns : -1;
      rc = ns <= INT32_MAX ? w * ns : 0;
    }
    rcnt[q] = rc;
  }
}

// The records of output vector v from record rb on: the G range of every
// stored S entry of the vector (inside split buckets [b0, b1), or the whole
// G vector for b0 < 0), and the entry's S value, in the order the product
// walk visits them. One wavefront, lanes over the entries.
template <int K>
__device__ __forceinline__ void vector_recs(const Plan &P, int64_t v, int32_t b0, int32_t b1, int64_t rb) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int l = lane();
  int64_t j = 0;
  const int64_t s1 = uload(P.ov_seg + v + 1);
  for (int64_t s = uload(P.ov_seg + v); s < s1; ++s) {
    const ProdDev d = uload(P.prods + uload(P.seg_prod + s));
    const int32_t t = uload(P.seg_svec + s);
    const int64_t e0 = uload(d.s_ptr + t), e1 = uload(d.s_ptr + t + 1);
    for (int64_t e = e0 + l; e < e1; e += kWave) {
      const int32_t k = gload(d.s_idx + e);
      const int32_t gt = d.gres ? gload(d.gres + e) : ((k >= 0 && k < d.g_nvec) ? k : -1);
      int64_t g = 0;
      int32_t len = 0;
      if (gt >= 0) {
        const int64_t p0 = gload(d.g_ptr + gt);
        if (b0 >= 0 && d.wsplit) {
          const int32_t *ws = d.wsplit + (int64_t)gt * (d.nsplit + 1);
          const int32_t a = gload(ws + b0);
          g = p0 + a;
          len = gload(ws + b1) - a;
        } else {
          g = p0;
          len = (int32_t)(gload(d.g_ptr + gt + 1) - p0);
        }
      }
      const int64_t x = rb + j + (e - e0);
      gstore(P.rec_gi + x, (int64_t)(d.g_idx + g));
      if (SR::kVal) gstore(P.rec_gv + x, (int64_t)((const T *)d.g_val + g));
      gstore(P.rec_len + x, len);
      if (SR::kVal) gstore((T *)P.rec_sv + x, gload((const T *)d.s_val + e));
    }
    j += e1 - e0;
  }
}

// One wavefront per heavy item with records (the G ranges inside the item's
// buckets).
template <int K>
__global__ void k_item_recs(Plan P) {
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t n = P.counters[kCtItems];
  for (int64_t it = wave; it < n; it += nwaves) {
    const ItemDev I = uload(P.items + it);
    if (I.rbase < 0) continue;
    vector_recs<K>(P, I.v, I.b0, I.b1, I.rbase);
  }
}

// The mid-tier vector at record position p: the mid list, then the small list.
__device__ __forceinline__ int32_t mid_pos_vector(const Plan &P, int64_t nm, int64_t p) {
  return p < nm ? P.mid_list[p] : P.small_list[p - nm];
}

// Records of the mid-tier vectors: per position i (mid list, then small
// list) the vector's stored S entries (mcnt, scanned into mbase), placed
// after the heavy items' records (whose total is *heavy_total).
__global__ void k_mid_rec_count(Plan P, int64_t cap, int64_t *mcnt) {
  const int64_t nm = P.counters[kCtMid];
  const int64_t np = nm + P.counters[kCtSmall];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t ns = 0;
    if (i < np) {
      const int32_t v = mid_pos_vector(P, nm, i);
      for (int64_t s = P.ov_seg[v]; s < P.ov_seg[v + 1]; ++s) {
        const ProdDev &d = P.prods[P.seg_prod[s]];
        const int32_t t = P.seg_svec[s];
        ns += d.s_ptr[t + 1] - d.s_ptr[t];
      }
    }
    mcnt[i] = ns <= INT32_MAX ? ns : 0;
  }
}

// A mid vector keeps its records when all of them fit the workspace.
__global__ void k_mid_rec_base(Plan P, int64_t cap, const int64_t *heavy_total, const int64_t *mcnt,
                               const int64_t *mbase, int64_t *mid_rb, int32_t *mid_nrec) {
  const int64_t np = P.counters[kCtMid] + P.counters[kCtSmall];
  const int64_t h = *heavy_total;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = h + mbase[i];
    const bool ok = i < np && mcnt[i] > 0 && r0 + mcnt[i] <= P.rec_cap;
    mid_rb[i] = ok ? r0 : -1;
    mid_nrec[i] = ok ? (int32_t)mcnt[i] : 0;
  }
}

// One wavefront per mid-tier vector with records (whole G vectors).
template <int K>
__global__ void k_mid_recs(Plan P) {
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t nm = P.counters[kCtMid];
  const int64_t n = nm + P.counters[kCtSmall];
  for (int64_t i = wave; i < n; i += nwaves) {
    const int64_t rb = uload(P.mid_rb + i);
    if (rb < 0) continue;
    vector_recs<K>(P, i < nm ? uload(P.mid_list + i) : uload(P.small_list + (i - nm)), -1, -1, rb);
  }
}

// Per-group totals after the scans of counts (ov_off) and non-empty flags (nzpos).
__global__ void k_group_totals(GroupDev *groups, int32_t ngroup, const int64_t *ov_off, const int64_t *nzpos,
                               int64_t *gstat) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroup) return;
  GroupDev &G = groups[g];
  G.nnz_base = ov_off[G.ov_begin];
  G.nz_base = nzpos[G.ov_begin];
  gstat[g * kStCount + kStNnz] = ov_off[G.ov_end] - G.nnz_base;
  gstat[g * kStCount + kStNvec] = nzpos[G.ov_end] - G.nz_base;
  gstat[g * kStCount + kStOutVec] = G.ov_end - G.ov_begin;
}

// ---- output pointers --------------------------------------------------------
// CSR/CSC output: ptr[j] for every major id j of every group (dense range
// dbase[g] .. dbase[g] + major_g inclusive).
__global__ void k_emit_ptr_dense(Plan P, const int64_t *pbase, int32_t ngroup, int64_t ntot) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < ntot; x += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = ngroup - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (pbase[mid] <= x) lo = mid; else hi = mid - 1;
    }
    const GroupDev &G = P.groups[lo];
    const OutDev &O = P.outs[lo];
    int64_t j = x - pbase[lo];
    int64_t a = G.ov_begin, b = G.ov_end;  // first v with ov_id >= j
    while (a < b) {
      int64_t mid = a + ((b - a) >> 1);
      if (P.ov_id[mid] < j) a = mid + 1; else b = mid;
    }
    O.ptr[j] = P.ov_off[a] - G.nnz_base;
  }
}

// Doubly compressed output: JC/CP of the non-empty vectors.
__global__ void k_emit_ptr_doubly(Plan P, const int64_t *nzpos, int32_t ngroup) {
  const int64_t nov = P.counters[kCtNov];
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= nov; v += (int64_t)gridDim.x * blockDim.x) {
    if (v == nov) {
      for (int32_t g = 0; g < ngroup; ++g) {
        const GroupDev &G = P.groups[g];
        P.outs[g].ptr[nzpos[G.ov_end] - G.nz_base] = P.ov_off[G.ov_end] - G.nnz_base;
      }
      continue;
    }
    if (P.ov_cnt[v] == 0) continue;
    const int32_t g = uload(P.ov_group + v);
    const GroupDev &G = P.groups[g];
    int64_t pos = nzpos[v] - G.nz_base;
    P.outs[g].vid[pos] = P.ov_id[v];
    P.outs[g].ptr[pos] = P.ov_off[v] - G.nnz_base;
  }
}

// ---- output table -----------------------------------------------------------
// The output descriptors of up to kOutChunk groups travel in the kernel's
// arguments, so a launch recorded in a HIP graph carries its own table and
// later calls with other outputs cannot redirect its replays.
constexpr int kOutChunk = 24;
struct OutChunk {
  OutDev o[kOutChunk];
};

__global__ void k_set_outs(OutDev *table, int32_t first, int32_t n, OutChunk chunk) {
  const int i = threadIdx.x;
  if (i < n) table[first + i] = chunk.o[i];
}

// ---- operand validation -----------------------------------------------------
__global__ void k_validate(const int64_t *ptr, const int32_t *vid, const int32_t *idx, int64_t nvec, int64_t nnz,
                           int64_t major, int64_t minor, int32_t doubly, int64_t *bad) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nvec; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = ptr[t], b = ptr[t + 1];
    bool ok = a >= 0 && b >= a && b <= nnz;
    if (t == 0) ok = ok && a == 0;
    if (t == nvec - 1) ok = ok && b == nnz;
    if (doubly) {
      ok = ok && b > a && vid[t] >= 0 && vid[t] < major;
      if (t > 0) ok = ok && vid[t - 1] < vid[t];
    }
    if (ok) {
      for (int64_t e = a; e < b; ++e) {
        int32_t i = idx[e];
        if (i < 0 || i >= minor || (e > a && idx[e - 1] >= i)) {
          ok = false;
          break;
        }
      }
    }
    if (!ok) atomicAdd((unsigned long long *)bad, 1ull);
  }
}

}  // namespace sg
