// Device-side format utilities (paper, Sections 2.2 and 2.3: CSR/CSC and the
// doubly compressed DCSC whose JC lists only the non-empty columns; Section
// 2.4: the transpose that turns a row-major operand into a column-major one).
//
//   triples -> compressed: the triples are ordered by (major, minor) with a
//       stable least-significant-digit radix sort, so that repeated positions
//       stay in list order; each run of one position is then combined with
//       the semiring's add as a left fold in that order, and the pointers
//       (and, doubly compressed, the ids of the non-empty vectors) follow
//       from run heads and scans.
//   format change: between orientations the entries are re-ordered by their
//       minor id with the same stable sort (the storage of M^T); entries of
//       one new vector then keep ascending old major ids, which are their new
//       minor ids. Within one orientation only the pointer array changes.
//
// The radix sort moves 8 bits per pass. A tile of 4096 keys (256 threads, 16
// rounds of 256) counts its digits in LDS; a scan over (digit, tile) gives
// every tile its output offset per digit; the scatter pass ranks each key
// among the equal digits before it in the tile (ballots inside a wavefront,
// per-wavefront counts across the four wavefronts, a running count per digit
// across rounds), so keys with equal digits keep their input order.
#pragma once

#include "sg_device.h"

namespace sg {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kSortWaves = kSortThreads / kWave;

// Digit counts of one tile: hist[d * ntile + tile].
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t *keys, int64_t n, int shift, int64_t ntile,
                                                              int64_t *hist) {
  __shared__ uint32_t cnt[256];
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    if (i < n) atomicAdd(&cnt[(uint32_t)(gload(keys + i) >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * ntile + blockIdx.x] = cnt[tid];
}

// Stable scatter of one pass: the key at input position i goes to
// off[d * ntile + tile] + (keys of digit d before it in the tile). PAY moves an
// int32 payload, VB the bytes of a value payload (0, 4 or 8).
template <int VB, bool PAY>
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint64_t *kin, const int32_t *pin, const void *vin,
                                                                 int64_t n, int shift, int64_t ntile, const int64_t *off,
                                                                 uint64_t *kout, int32_t *pout, void *vout) {
  typedef typename std::conditional<VB == 8, uint64_t, uint32_t>::type V;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kSortWaves][256];
  __shared__ int64_t boff[256];
  const int tid = threadIdx.x, w = tid / kWave, l = lane();
  run[tid] = 0;
  boff[tid] = off[(int64_t)tid * ntile + blockIdx.x];
  const uint64_t lt = (1ull << l) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int x = 0; x < kSortWaves; ++x) wcnt[x][tid] = 0;
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < n;
    const uint64_t key = valid ? gload(kin + i) : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    __syncthreads();  // the clears and the previous round's running counts are visible
    // lanes of this wavefront holding the same digit: one ballot per digit bit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t before = run[d];
      for (int x = 0; x < w; ++x) before += wcnt[x][d];
      const int64_t pos = boff[d] + before + rank;
      gstore(kout + pos, key);
      if (PAY) gstore(pout + pos, gload(pin + i));
      if (VB) gstore((V *)vout + pos, gload((const V *)vin + i));
    }
    uint32_t tot = 0;
#pragma unroll
    for (int x = 0; x < kSortWaves; ++x) tot += wcnt[x][tid];
    __syncthreads();  // every read of run and wcnt of this round is done
    run[tid] += tot;
  }
}

// Keys of a triple list: major * minor_dim + minor (row-major: major = row).
// Triples outside the matrix are counted in *bad.
__global__ void k_coo_keys(const int32_t *rows, const int32_t *cols, int64_t n, int32_t row_major, int64_t nrows,
                           int64_t ncols, uint64_t *keys, int64_t *bad) {
  const int64_t minor_dim = row_major ? ncols : nrows;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = gload(rows + i), c = gload(cols + i);
    if (r < 0 || r >= nrows || c < 0 || c >= ncols) {
      atomicAdd((unsigned long long *)bad, 1ull);
      gstore(keys + i, (uint64_t)0);
      continue;
    }
    const int64_t maj = row_major ? r : c, mnr = row_major ? c : r;
    gstore(keys + i, (uint64_t)(maj * minor_dim + mnr));
  }
}

// Triple lists of at most kCooSmall entries are compressed by one workgroup
// (a request's frontier, say): keys and their list positions packed into one
// 64-bit LDS word, a bitonic sort in LDS, then run and vector heads and
// their scans, written where the general path's sort, head and scan kernels
// leave them. One launch instead of about fifteen.
constexpr int kCooSmall = 4096;
constexpr int kCooSmallBits = 12;  // list positions < kCooSmall
constexpr int kCooSmallThreads = 1024;

__global__ void __launch_bounds__(kCooSmallThreads) k_coo_small(const int32_t *rows, const int32_t *cols,
                                                                const void *vals, int64_t n, int32_t row_major,
                                                                int64_t nrows, int64_t ncols, int vb,
                                                                uint64_t *keys_out, void *vals_out, int64_t *head,
                                                                int64_t *vhead, int64_t *upos, int64_t *vpos,
                                                                int64_t *bad) {
  __shared__ uint64_t sk[kCooSmall];
  __shared__ int64_t scratch[kMaxWaves + 1];
  const int t = threadIdx.x, nt = blockDim.x;
  const int64_t minor_dim = row_major ? ncols : nrows;
  const uint64_t md = minor_dim > 0 ? (uint64_t)minor_dim : 1;  // for the vector heads
  int np = 2;
  while (np < n) np <<= 1;
  // (key << 12 | position): equal keys keep their list order; padding sorts last
  for (int i = t; i < np; i += nt) {
    uint64_t e = ~0ull;
    if (i < n) {
      const int64_t r = gload(rows + i), c = gload(cols + i);
      uint64_t key = 0;
      if (r < 0 || r >= nrows || c < 0 || c >= ncols) {
        atomicAdd((unsigned long long *)bad, 1ull);
      } else {
        const int64_t maj = row_major ? r : c, mnr = row_major ? c : r;
        key = (uint64_t)(maj * minor_dim + mnr);
      }
      e = (key << kCooSmallBits) | (uint64_t)i;
    }
    sk[i] = e;
  }
  __syncthreads();
  for (int k = 2; k <= np; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < np; i += nt) {
        const int x = i ^ j;
        if (x > i) {
          const uint64_t a = sk[i], b = sk[x];
          const bool up = (i & k) == 0;
          if (up ? a > b : a < b) {
            sk[i] = b;
            sk[x] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // sorted keys and values, run heads and vector heads; thread t takes the
  // consecutive positions [t * per, (t + 1) * per) for the scans
  const int per = (int)((n + nt - 1) / nt);
  const int i0 = t * per < n ? t * per : (int)n;
  const int i1 = i0 + per < n ? i0 + per : (int)n;
  int64_t nh = 0, nv = 0;
  for (int i = i0; i < i1; ++i) {
    const uint64_t e = sk[i];
    const uint64_t key = e >> kCooSmallBits;
    const int src = (int)(e & (uint64_t)(kCooSmall - 1));
    gstore(keys_out + i, key);
    if (vb == 8) gstore((uint64_t *)vals_out + i, gload((const uint64_t *)vals + src));
    else if (vb == 4) gstore((uint32_t *)vals_out + i, gload((const uint32_t *)vals + src));
    const uint64_t prev = i > 0 ? sk[i - 1] >> kCooSmallBits : ~0ull;
    const bool h = i == 0 || key != prev;
    const bool vh = h && (i == 0 || key / md != prev / md);
    gstore(head + i, (int64_t)h);
    gstore(vhead + i, (int64_t)vh);
    nh += h;
    nv += vh;
  }
  int64_t th, tv;
  int64_t ph = block_excl_scan(nh, scratch, &th);
  int64_t pv = block_excl_scan(nv, scratch, &tv);
  for (int i = i0; i < i1; ++i) {
    gstore(upos + i, ph);
    gstore(vpos + i, pv);
    const uint64_t key = sk[i] >> kCooSmallBits;
    const uint64_t prev = i > 0 ? sk[i - 1] >> kCooSmallBits : ~0ull;
    const bool h = i == 0 || key != prev;
    ph += h;
    pv += h && (i == 0 || key / md != prev / md);
  }
  if (t == 0) {
    gstore(upos + n, th);
    gstore(vpos + n, tv);
    gstore(bad + 1, th);  // beside the bad-triple count, for one readback
    gstore(bad + 2, tv);
  }
}

// Run heads of sorted keys (a new position) and vector heads (a new major).
__global__ void k_key_heads(const uint64_t *keys, int64_t n, uint64_t minor_dim, int64_t *head, int64_t *vhead) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = gload(keys + i);
    const uint64_t p = i > 0 ? gload(keys + i - 1) : ~0ull;
    const bool h = i == 0 || k != p;
    gstore(head + i, (int64_t)h);
    gstore(vhead + i, (int64_t)(h && (i == 0 || k / minor_dim != p / minor_dim)));
  }
}

// Entries of the compressed output: one per run of equal keys, its value the
// left fold of the run's values in their (stable) order. Plain output counts
// the entries per major id (cnt, scanned into ptr afterwards); doubly
// compressed output writes vid and ptr at the vector heads.
template <int K>
__global__ void k_coo_emit(const uint64_t *keys, const void *vals, int64_t n, uint64_t minor_dim, const int64_t *head,
                           const int64_t *upos, const int64_t *vhead, const int64_t *vpos, int32_t doubly,
                           int32_t *idx, void *val, int32_t *vid, int64_t *ptr, int64_t *cnt) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!gload(head + i)) continue;
    const uint64_t k = gload(keys + i);
    const int64_t u = gload(upos + i);
    const uint64_t maj = k / minor_dim;
    gstore(idx + u, (int32_t)(k - maj * minor_dim));
    if (SR::kVal) {
      T acc = gload((const T *)vals + i);
      for (int64_t j = i + 1; j < n && gload(keys + j) == k; ++j) acc = SR::add(acc, gload((const T *)vals + j));
      gstore((T *)val + u, acc);
    }
    if (doubly) {
      if (gload(vhead + i)) {
        const int64_t v = gload(vpos + i);
        gstore(vid + v, (int32_t)maj);
        gstore(ptr + v, u);
      }
    } else {
      atomicAdd((unsigned long long *)(cnt + maj), 1ull);
    }
  }
}

// ptr[nvec] = nnz for a doubly compressed output (or an empty one's ptr[0] = 0).
__global__ void k_set_i64(int64_t *p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---- format change of a canonical matrix ---------------------------------
// Stored vector of entry e: the last t with ptr[t] <= e (binary search).
__device__ __forceinline__ int64_t vector_of(const int64_t *ptr, int64_t nvec, int64_t e) {
  int64_t lo = 0, hi = nvec - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (gload(ptr + mid) <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Entries per major id of a doubly compressed matrix (cnt zeroed before).
__global__ void k_vec_counts(const int64_t *ptr, const int32_t *vid, int64_t nvec, int64_t *cnt) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nvec; t += (int64_t)gridDim.x * blockDim.x)
    gstore(cnt + gload(vid + t), gload(ptr + t + 1) - gload(ptr + t));
}

// Entries per key (a histogram of the sorted new majors; cnt zeroed before).
__global__ void k_key_counts(const uint64_t *keys, int64_t n, int64_t *cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long *)(cnt + gload(keys + i)), 1ull);
}

// Non-empty flags of the vectors of a plain compressed matrix.
__global__ void k_vec_nonempty(const int64_t *ptr, int64_t nvec, int64_t *flag) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nvec; t += (int64_t)gridDim.x * blockDim.x)
    gstore(flag + t, (int64_t)(gload(ptr + t + 1) > gload(ptr + t)));
}

// Doubly compressed pointers of a plain compressed matrix (ids shifted to 0).
__global__ void k_compress_ptr(const int64_t *ptr, int64_t nvec, const int64_t *flag, const int64_t *pos,
                               int32_t *vid_out, int64_t *ptr_out) {
  const int64_t p0 = gload(ptr);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nvec; t += (int64_t)gridDim.x * blockDim.x) {
    if (!gload(flag + t)) continue;
    const int64_t v = gload(pos + t);
    gstore(vid_out + v, (int32_t)t);
    gstore(ptr_out + v, gload(ptr + t) - p0);
  }
}

// Plain copy of n elements of `bytes` bytes each (4 or 8), in 4-byte words.
__global__ void k_copy_words(const uint32_t *src, uint32_t *dst, int64_t nwords) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
    gstore(dst + i, gload(src + i));
}

// Doubly compressed pointers from run heads of sorted new-major keys.
__global__ void k_heads_to_doubly(const uint64_t *keys, int64_t n, const int64_t *head, const int64_t *hpos,
                                  int32_t *vid_out, int64_t *ptr_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!gload(head + i)) continue;
    const int64_t v = gload(hpos + i);
    gstore(vid_out + v, (int32_t)gload(keys + i));
    gstore(ptr_out + v, i);
  }
}

}  // namespace sg
