// Device-side types and wavefront helpers of the local sparse product library.
//
// Terminology used throughout the kernels (column-major view; the row-major
// case is the same on the transposes):
//   S  the streamed operand, whose vectors define the output vectors
//      (B for C = A B in CSC/DCSC, A in CSR/DCSR),
//   G  the gathered operand, whose vector k is fetched for every stored
//      entry (k, s) of an S vector (A in CSC/DCSC, B in CSR/DCSR).
// C(:, j) = (+)_{(k, s) in S(:, j)} G(:, k) (x) s, the column-by-column
// formulation (paper, Section 2.1). The four semirings' multiplies are all
// commutative, so g (x) s equals the paper's A(i,k) (x) B(k,j) in both
// orientations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sg_spgemm.h"

namespace sg {

constexpr int kWave = 64;
constexpr int kXcds = 8;           // dies of an MI355X, each with its own L2
constexpr int kMaxWaves = 16;  // 1024 threads per workgroup at most
constexpr int kBlockMax = 1024;    // threads per workgroup of the mid/heavy/batched kernels
// SG_CHECK=1 builds the invariant-checking variant of the library: every
// persistent kernel verifies after each work item that its dynamic LDS is
// back to all-zero bits, and every numeric tier compares the entries it
// writes with the exact count the symbolic phase planned. Violations are
// counted in the plan's counters (read with sg_plan_check); the arithmetic
// and the results are those of the normal build.
#ifndef SG_CHECK
#define SG_CHECK 0
#endif
#ifndef SG_WAVES_PER_SIMD
#define SG_WAVES_PER_SIMD 4
#endif
constexpr int kWavesPerSimd = SG_WAVES_PER_SIMD;  // occupancy the register budget is sized for

// One product A_p (x) B_p, in S/G terms, as the kernels see it.
struct ProdDev {
  const int64_t *s_ptr;
  const int32_t *s_vid;  // major ids of S vectors (doubly compressed) or null
  const int32_t *s_idx;
  const void *s_val;
  int64_t s_nvec;
  const int64_t *g_ptr;
  const int32_t *g_vid;  // doubly compressed G: ids of stored vectors, else null
  const int32_t *g_idx;
  const void *g_val;
  int64_t g_nvec;
  int64_t g_major;       // number of vectors of G as a matrix (its major dimension)
  const int32_t *aux;    // AUX index of a doubly compressed G (Section 2.3), else null
  int64_t aux_chunk;     // columns per AUX chunk
  int64_t aux_n;         // number of AUX chunks
  int32_t *gres;         // per S entry: resolved G vector (doubly compressed G only)
  int32_t *wsplit;       // per G vector: nsplit + 1 offsets of the split buckets, or null
  int32_t group;
  int32_t nsplit;        // split buckets of this product's group
};

// One output C_g.
struct GroupDev {
  int64_t minor;         // minor dimension of C_g (its output id range)
  int64_t major;         // major dimension of C_g
  int32_t nsplit;        // split buckets of `sw` ids covering [0, minor)
  int32_t sw;            // split bucket width (a multiple of 32)
  int32_t mode;          // heavy tier: 0 dense windows of one bucket, 1 rank windows of several buckets
  int32_t mid_ok;        // largest mid-tier vector of this group (0: the mid tier does not fit)
  int32_t rank_cap;      // mode 1: LDS of one window in value slots ({bits, prefix} words plus values)
  int32_t rank_wb;       // mode 1: most buckets one window may span
  int32_t bpr;           // split buckets per XCD range (windows never cross a range)
  int32_t rank_wcost;    // mode 1: value slots taken by the {bits, prefix} words of one bucket
  int64_t ov_begin;      // first output vector of this group (device-filled)
  int64_t ov_end;
  int64_t nnz_base;      // global exclusive offset of the group's first entry
  int64_t nz_base;       // global count of non-empty vectors before the group
  // optional output mask: bit (i, j) of output vector j (its major id) and
  // output id i at mask[j * mask_stride + i / 32], bit i % 32; an entry is
  // kept where the bit is 0 (mask_comp = 1, e.g. not yet visited) or 1
  const uint32_t *mask;  // null: every entry is kept
  int64_t mask_stride;   // 32-bit words per output vector
  int32_t mask_comp;
  int32_t mask_pad;
};

// Mask word w (ids 32 w .. 32 w + 31) of output vector j: the bits of the ids
// the output keeps (all ones when the group has no mask).
__device__ __forceinline__ uint32_t keep_word(const uint32_t *mask, int64_t stride, int32_t comp, int64_t j, int64_t w) {
  if (mask == nullptr) return ~0u;
  const uint32_t m = *(const __attribute__((address_space(1))) uint32_t *)(mask + j * stride + w);
  return comp ? ~m : m;
}

// One heavy-tier item: the window of split buckets [b0, b1) of output
// vector v (position q in the heavy list) of group g, whose entries start at
// `pos` inside the group's output arrays.
// With entry records, rbase >= 0 is the first of the window's nrec records
// (one per stored S entry of v, over all of v's segments: the addresses of
// the entry's G slice inside the window and its S value), written once by
// the symbolic phase.
struct ItemDev {
  int32_t v;
  int32_t g;
  int32_t b0;
  int32_t b1;
  int64_t pos;
  int32_t q;
  int32_t nrec;
  int64_t rbase;
};

struct OutDev {
  int64_t *ptr;
  int32_t *vid;
  int32_t *idx;
  void *val;
  int32_t fmt;
  int32_t pad;
};

// Per-group statistics written by the symbolic kernels (int64 each).
enum GroupStat {
  kStFlops = 0,
  kStUb,
  kStMaxFlops,
  kStTiny,
  kStMid,
  kStHeavy,
  kStItems,
  kStNnz,
  kStNvec,
  kStOutVec,
  kStCount
};

// Global device counters (int64 each).
enum Counter {
  kCtNov = 0,      // output vectors
  kCtNseg,         // segments
  kCtTiny,         // tiny-tier vectors
  kCtMid,          // mid-tier vectors
  kCtHeavy,        // heavy-tier vectors
  kCtItems,        // heavy-tier (vector, window) items
  kCtQueue,        // work queue head of the persistent launch
  kCtQueueCount,   // work queue head of the persistent count launch
  kCtBad,          // validation failures
  kCtTierFlops,    // 3 entries: multiplications per tier
  kCtTierSent = kCtTierFlops + 3,  // 3 entries: streamed entries per tier
  kCtTierNnz = kCtTierSent + 3,    // 3 entries: output entries per tier
  kCtChkLds = kCtTierNnz + 3,      // invariant-check build: items that left LDS non-zero
  kCtChkCount,                     // invariant-check build: numeric counts that differ from the count pass
  kCtSmall,                        // mid-tier vectors run one per wavefront (the small list)
  kCtNum
};

// Everything a numeric or count kernel reads, passed by value.
struct Plan {
  const ProdDev *prods;
  const GroupDev *groups;
  const OutDev *outs;
  const int32_t *ov_id;
  const int32_t *ov_group;
  const int64_t *ov_seg;
  const int32_t *seg_prod;
  const int32_t *seg_svec;
  int64_t *ov_flops;
  int64_t *ov_cnt;
  const int64_t *ov_off;   // global exclusive scan of ov_cnt
  const int64_t *counters;
  const int32_t *tiny_list;
  const int32_t *mid_list;
  const int32_t *small_list;   // mid-tier vectors of at most kSmallMaxFlops products, one per wavefront
  const int32_t *heavy_list;
  const struct ItemDev *items;  // heavy (vector, window) items
  int32_t *bcnt;             // heavy vector q: entries per split bucket, at q * nbmax
  int32_t nbmax;             // largest nsplit of any group
  int32_t nrange;            // XCD ranges (8 per XCD share, or 1 when ranges are off)
  const int64_t *ibase;      // exclusive offsets of the heavy items by (range, vector)
  int64_t ibase_stride;      // entries per range in ibase
  uint32_t *hbits;           // kept id bitmaps of the first nkeep heavy vectors
  int64_t hstride;           // 32-bit words per kept bitmap
  int64_t nkeep;
  int64_t *rec_gi;           // entry records: address of the first G id of the entry's products in the window
  int64_t *rec_gv;           //   address of the first of their G values (valued semirings)
  int32_t *rec_len;          //   their count
  void *rec_sv;              //   the entry's S value
  int64_t rec_cap;           // records the workspace holds
  const int64_t *mid_rb;     // mid-tier vector at position p (mid list, then small list): its first record, or -1
  const int32_t *mid_nrec;   //   its record count (its stored S entries)
  int64_t *chk;              // invariant-check counters (the plan's counters; written only by SG_CHECK builds)
  int32_t mid_cap;           // max entries of a mid-tier vector
  int32_t mid_kind;          // 0 bitmap-rank, 1 hash
  int32_t lds_words;         // dynamic LDS size in 32-bit words
};

// ---------------------------------------------------------------------------
// Semiring traits. Every accumulator slot in LDS starts as all-zero bits,
// which must encode the additive identity: 0.0 for (+,*), and for (min,+)
// the slot holds INT32_MAX - v as an unsigned word, so the identity
// (INT32_MAX) is 0 and min becomes an unsigned max.
template <int K>
struct Sr;

template <>
struct Sr<SG_PLUS_TIMES_F64> {
  typedef double T;      // value type
  typedef double Slot;   // accumulator slot in LDS
  static constexpr bool kVal = true;
  __device__ static T mul(T s, T g) { return s * g; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static Slot enc(T v) { return v; }
  __device__ static T dec(Slot v) { return v; }
  __device__ static void acc(Slot *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <>
struct Sr<SG_PLUS_TIMES_F32> {
  typedef float T;
  typedef float Slot;
  static constexpr bool kVal = true;
  __device__ static T mul(T s, T g) { return s * g; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static Slot enc(T v) { return v; }
  __device__ static T dec(Slot v) { return v; }
  __device__ static void acc(Slot *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <>
struct Sr<SG_MIN_PLUS_I32> {
  typedef int32_t T;
  typedef uint32_t Slot;
  static constexpr bool kVal = true;
  __device__ static T mul(T s, T g) {
    if (s == INT32_MAX || g == INT32_MAX) return INT32_MAX;
    int64_t r = (int64_t)s + (int64_t)g;
    if (r > INT32_MAX) return INT32_MAX;
    if (r < INT32_MIN) return INT32_MIN;
    return (T)r;
  }
  __device__ static T add(T a, T b) { return a < b ? a : b; }
  __device__ static Slot enc(T v) { return (uint32_t)INT32_MAX - (uint32_t)v; }
  __device__ static T dec(Slot u) { return (T)((uint32_t)INT32_MAX - u); }
  __device__ static void acc(Slot *p, T v) {
    __hip_atomic_fetch_max(p, enc(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <>
struct Sr<SG_OR_AND_BOOL> {
  typedef uint32_t T;  // unused: pattern only
  typedef uint32_t Slot;
  static constexpr bool kVal = false;
  __device__ static T mul(T, T) { return 1u; }
  __device__ static T add(T, T) { return 1u; }
  __device__ static Slot enc(T v) { return v; }
  __device__ static T dec(Slot v) { return v; }
  __device__ static void acc(Slot *, T) {}
};

// ---------------------------------------------------------------------------
// Global-memory access through explicitly global pointers: pointers read out
// of descriptor structs are otherwise generic, and generic (flat) accesses
// share the LDS wait counter, so every LDS wait would also drain the loads.
#define SG_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gload(const T *p) {
  return *(const SG_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ void gstore(T *p, T v) {
  *(SG_GLOBAL T *)p = v;
}

// Wave-uniform reads of descriptors and index arrays that no running kernel
// writes (they are filled by earlier launches): through the constant address
// space a load with a wave-uniform address becomes a scalar load, issued once
// per wavefront and served by the scalar cache, instead of a chain of vector
// loads each followed by a wait. Read-only: nothing is ever stored this way.
#define SG_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ T uload(const T *p) {
  if constexpr (__is_scalar(T)) {
    return *(const SG_CONST T *)p;
  } else {  // descriptor structs: word by word (merged into wide scalar loads)
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T out;
    uint32_t *o = (uint32_t *)&out;
    const SG_CONST uint32_t *q = (const SG_CONST uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = q[i];
    return out;
  }
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Marks a value the caller knows to be wave-uniform (lane 0's copy is taken).
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Inclusive sum over lanes 0..l, on the VALU with DPP: row shifts by 1, 2,
// 4 and 8 scan each 16-lane row (lanes shifted in from outside the row read
// 0), then the last lane of each row is added to the next row and the last
// lane of the first half to the second half. Every lane must be active.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1 and 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x) {
  const int l = lane();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t t = __shfl_up(x, d, kWave);
    if (l >= d) x += t;
  }
  return x;
}


// Uniform read of lane o's value (o is wave-uniform).
__device__ __forceinline__ int read_lane(int x, int o) { return __builtin_amdgcn_readlane(x, o); }

// Lane l receives lane (l xor j)'s x, for a power of two j that is a
// constant once loops are unrolled: quad permutes (1, 2) and row shifts
// (4, 8) of DPP and the 16- and 32-lane swaps of gfx950 (16, 32), all on
// the VALU, so a sorting network moves no data through LDS. Every lane of
// the wavefront must be active.
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, int j) {
  const int l = lane();
  const int v = (int)x;
  switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    case 4: {
      const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, false);  // row_shl:4, lane l + 4
      const int dn = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, false);  // row_shr:4, lane l - 4
      return (uint32_t)((l & 4) ? dn : up);
    }
    case 8: {
      const int up = __builtin_amdgcn_mov_dpp(v, 0x108, 0xF, 0xF, false);  // row_shl:8
      const int dn = __builtin_amdgcn_mov_dpp(v, 0x118, 0xF, 0xF, false);  // row_shr:8
      return (uint32_t)((l & 8) ? dn : up);
    }
    case 16: {
      // first result: even rows copied over the odd ones; second: odd rows over the even ones
      const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
      return (l & 16) ? r[0] : r[1];
    }
    case 32: {
      // first result: the low half in both halves; second: the high half in both
      const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
      return (l & 32) ? r[0] : r[1];
    }
    default: return (uint32_t)__shfl_xor(v, j, kWave);
  }
}
__device__ __forceinline__ int32_t xor_lane(int32_t x, int j) { return (int32_t)xor_lane((uint32_t)x, j); }
__device__ __forceinline__ uint64_t xor_lane(uint64_t x, int j) {
  return ((uint64_t)xor_lane((uint32_t)(x >> 32), j) << 32) | xor_lane((uint32_t)x, j);
}
__device__ __forceinline__ double xor_lane(double x, int j) {
  return __longlong_as_double((long long)xor_lane((uint64_t)__double_as_longlong(x), j));
}
__device__ __forceinline__ float xor_lane(float x, int j) {
  return __uint_as_float(xor_lane((uint32_t)__float_as_uint(x), j));
}

// One compare-exchange of a bitonic step across lanes: the lane keeps the
// smaller of its key and its partner's key pk when keep_min, else the larger,
// with the value that goes with it. The choice is two selects: written as a
// branch on the divergent comparison, the compiler emits an exec-mask diamond
// per step.
template <class KT, class T>
__device__ __forceinline__ void cmp_exchange(KT &key, T &val, KT pk, T pv, bool keep_min) {
  const bool lt = pk < key, gt = key < pk;
  const bool take = (keep_min & lt) | (!keep_min & gt);
  key = take ? pk : key;
  val = take ? pv : val;
}

// One DPP move of a 64-bit value (both halves with the same control);
// lanes without a source lane, or in rows outside ROWS, get `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t old, uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)old, (int)(uint32_t)x, CTRL, ROWS, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(old >> 32), (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_any(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_any(int32_t x) { return (int32_t)dpp_any<CTRL, ROWS>((uint32_t)x); }
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_any(float x) { return __uint_as_float(dpp_any<CTRL, ROWS>(__float_as_uint(x))); }
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_any(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return __longlong_as_double((long long)dpp64<CTRL, ROWS>(b, b));
}

// Lane l + 1's key (lane 63 gets ~key, which differs from its own).
__device__ __forceinline__ uint64_t next_lane_key(uint64_t key) { return dpp64<0x130, 0xF>(~key, key); }  // wave_shl:1

// Inclusive prefix, with the semiring's add, over each run of equal keys
// (runs are contiguous: the keys are sorted): lane l ends with the sum of
// its run's lanes up to l, so a run's last lane holds the run's total.
// Steps of 1, 2, 4 and 8 lanes inside each 16-lane row, then lane 15 of a
// row is added into the next row and lane 31 into the upper half, each
// where the key still matches (a lane without a source sees ~key). All on
// the VALU; every lane must be active.
template <class SR, class T>
__device__ __forceinline__ T seg_prefix(uint64_t key, T val) {
  const uint64_t miss = ~key;
#define SG_SEG_STEP(CTRL, ROWS)                                 \
  {                                                             \
    const uint64_t k = dpp64<CTRL, ROWS>(miss, key);            \
    const T v = dpp_any<CTRL, ROWS>(val);                       \
    if (k == key) val = SR::add(val, v);                        \
  }
  SG_SEG_STEP(0x111, 0xF)  // row_shr:1
  SG_SEG_STEP(0x112, 0xF)  // row_shr:2
  SG_SEG_STEP(0x114, 0xF)  // row_shr:4
  SG_SEG_STEP(0x118, 0xF)  // row_shr:8
  SG_SEG_STEP(0x142, 0xA)  // row_bcast:15 into rows 1 and 3
  SG_SEG_STEP(0x143, 0xC)  // row_bcast:31 into rows 2 and 3
#undef SG_SEG_STEP
  return val;
}

// Butterfly reductions over the wavefront (every lane gets the result).
__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += (int64_t)xor_lane((uint64_t)x, d);
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += xor_lane((int32_t)x, d);
  return x;
}

__device__ __forceinline__ int64_t wave_max64(int64_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const int64_t t = (int64_t)xor_lane((uint64_t)x, d);
    x = t > x ? t : x;
  }
  return x;
}
__device__ __forceinline__ int64_t read_lane64(int64_t x, int o) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, o);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), o);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double read_lane_f64(double x, int o) {
  return __longlong_as_double(read_lane64(__double_as_longlong(x), o));
}
__device__ __forceinline__ float read_lane_f32(float x, int o) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), o));
}
__device__ __forceinline__ int32_t read_lane_val(int32_t x, int o) { return read_lane(x, o); }
__device__ __forceinline__ uint32_t read_lane_val(uint32_t x, int o) { return (uint32_t)read_lane((int)x, o); }
__device__ __forceinline__ double read_lane_val(double x, int o) { return read_lane_f64(x, o); }
__device__ __forceinline__ float read_lane_val(float x, int o) { return read_lane_f32(x, o); }

// Smallest lane l with P[l] > f, for an inclusive prefix P held one per lane
// (every lane must execute this call).
__device__ __forceinline__ int owner_of(int P, int f) {
  int lo = 0;
#pragma unroll
  for (int step = kWave / 2; step > 0; step >>= 1) {
    int pc = __shfl(P, lo + step - 1, kWave);
    if (pc <= f) lo += step;
  }
  return lo;
}

// Exclusive scan across the workgroup; `scratch` holds kMaxWaves + 1 int64.
// Every thread sums the wavefront totals before its own wavefront (at most
// 16 broadcast reads) instead of one thread scanning them between two
// barriers; the last barrier keeps `scratch` intact until all have read it.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *scratch, int64_t *total) {
  const int l = lane();
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int64_t inc = wave_incl_scan64(x);
  if (l == kWave - 1) scratch[w] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    const int64_t t = scratch[i];
    before += i < w ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();
  return before + inc - x;
}

__device__ __forceinline__ int64_t block_sum(int64_t x, int64_t *scratch) {
  int64_t total;
  block_excl_scan(x, scratch, &total);
  return total;
}

// Locate vector k of a doubly compressed G via its AUX index; -1 if absent.
__device__ __forceinline__ int32_t aux_find(const ProdDev &d, int64_t k) {
  if (k < 0 || k >= d.g_major) return -1;
  int64_t c = k / d.aux_chunk;
  int32_t lo = gload(d.aux + c), hi = gload(d.aux + c + 1);
  const int32_t end = hi;
  while (lo < hi) {
    int32_t mid = lo + ((hi - lo) >> 1);
    if (gload(d.g_vid + mid) < k) lo = mid + 1; else hi = mid;
  }
  return (lo < end && gload(d.g_vid + lo) == k) ? lo : -1;
}

}  // namespace sg
