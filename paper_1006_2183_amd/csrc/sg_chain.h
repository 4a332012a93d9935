// Fused chain product C = G2 (G1 S) without materialising the intermediate
// product (paper, Section 8: triple products such as the Galerkin R A P of
// multigrid setup are the next step beyond one SpGEMM).
//
// Column-major C = R A P: S = P (its columns define C's columns), G1 = A,
// G2 = R; row-major C = R A P: S = R (its rows define C's rows), G1 = A,
// G2 = P. For an output vector j,
//   stage 1: T = (+)_{(l, s) in S(:, j)} G1(:, l) (x) s   (one vector of G1 S),
//   stage 2: C(:, j) = (+)_{(k, t) in T} G2(:, k) (x) t,
// and T lives only in registers (tiny tier: both stages have at most 64
// multiplications, one wavefront sorts and merges each stage) or in LDS
// (mid tier: stage 1 accumulates in an LDS hash whose entries are then the
// streamed entries of stage 2, which accumulates in a second LDS hash and is
// sorted there). The result equals the two-call product G2 (G1 S): T is
// merged before stage 2, exactly the intermediate the two calls would write.
#pragma once

#include "sg_tiers.h"

namespace sg {

// One chain product, in S/G1/G2 terms (plain compressed operands).
struct ChainDev {
  const int64_t *s_ptr;
  const int32_t *s_idx;
  const void *s_val;
  int64_t s_nvec;
  const int64_t *g1_ptr;  // vector l of G1 for every id l of S
  const int32_t *g1_idx;
  const void *g1_val;
  int64_t g1_nvec;
  const int64_t *g2_ptr;  // vector k of G2 for every id k of G1
  const int32_t *g2_idx;
  const void *g2_val;
  int64_t g2_nvec;
  int64_t t_minor;        // id range of the intermediate (minor dimension of G1)
  int32_t group;
  int32_t pad;
};

// Per output vector: stage-1 multiplications (ov_flops) and the unmerged
// fused count sum_{(l, s)} sum_{k in G1(:, l)} nnz(G2(:, k)), an upper bound
// of stage 2's (chain_bound); tiers by both. One lane per vector; a lane
// loads four S entries' G1 pointer pairs at a time and eight G1 ids' G2
// pointer pairs at a time, so its chain of dependent loads is about two per
// eight multiplications rather than two per multiplication. The group totals
// are summed over the wavefront before their atomics.
__global__ void k_chain_flops(Plan P, const ChainDev *chains, BinParams bp, int32_t mid_cap1, int32_t mid_cap2,
                              int64_t *bound, int64_t *gstat, int64_t *counters, int32_t *tiny, int32_t *mid) {
  constexpr int kE = 4, kQ = 8;
  const int64_t nov = counters[kCtNov];
  for (int64_t v0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave * kWave; v0 < nov;
       v0 += ((int64_t)gridDim.x * blockDim.x) / kWave * kWave) {
    const int64_t v = v0 + lane();
    const bool valid = v < nov;
    int64_t f1 = 0, fu = 0;
    int tier = -1;
    int32_t g = -1;
    int64_t ubv = 0;
    if (valid) {
      const int32_t p = gload(P.seg_prod + v), t = gload(P.seg_svec + v);
      const ChainDev *C = chains + p;
      const int32_t *s_idx = gload(&C->s_idx);
      const int64_t *g1_ptr = gload(&C->g1_ptr);
      const int32_t *g1_idx = gload(&C->g1_idx);
      const int64_t *g2_ptr = gload(&C->g2_ptr);
      const int64_t g1_nvec = gload(&C->g1_nvec), g2_nvec = gload(&C->g2_nvec);
      const int64_t *s_ptr = gload(&C->s_ptr);
      g = gload(&C->group);
      const int64_t es = gload(s_ptr + t), ee = gload(s_ptr + t + 1);
      for (int64_t e = es; e < ee; e += kE) {
        int32_t li[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) li[j] = e + j < ee ? gload(s_idx + e + j) : -1;
        int64_t a0[kE], a1[kE];
#pragma unroll
        for (int j = 0; j < kE; ++j) {
          const bool ok = li[j] >= 0 && li[j] < g1_nvec;
          a0[j] = ok ? gload(g1_ptr + li[j]) : 0;
          a1[j] = ok ? gload(g1_ptr + li[j] + 1) : 0;
        }
#pragma unroll
        for (int j = 0; j < kE; ++j) {
          f1 += a1[j] - a0[j];
          for (int64_t q = a0[j]; q < a1[j]; q += kQ) {
            int32_t k[kQ];
#pragma unroll
            for (int u = 0; u < kQ; ++u) k[u] = q + u < a1[j] ? gload(g1_idx + q + u) : -1;
            int64_t b0[kQ], b1[kQ];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
              const bool ok = k[u] >= 0 && k[u] < g2_nvec;
              b0[u] = ok ? gload(g2_ptr + k[u]) : 0;
              b1[u] = ok ? gload(g2_ptr + k[u] + 1) : 0;
            }
#pragma unroll
            for (int u = 0; u < kQ; ++u) fu += b1[u] - b0[u];
          }
        }
      }
      gstore(P.ov_flops + v, f1);
      gstore(bound + v, fu);
      const int64_t minor = P.groups[g].minor;
      const int64_t t_minor = gload(&C->t_minor);
      const int64_t ub1 = f1 < t_minor ? f1 : t_minor, ub2 = fu < minor ? fu : minor;
      if (fu == 0) tier = -1;
      else if (f1 <= bp.tiny_max && fu <= bp.tiny_max && bp.force != 1) tier = 0;
      else if (ub1 <= mid_cap1 && ub2 <= mid_cap2) tier = 1;
      else tier = 2;  // beyond the fused tiers: reported, the plan is refused
      ubv = ub2;
    }
    const uint64_t bad = __ballot(valid && tier == 2);
    if (bad && lane() == 0) atomicAdd((unsigned long long *)&counters[kCtBad], (unsigned long long)__popcll(bad));
    // group totals, one atomic per group present in the wavefront
    const bool counted = valid && tier >= 0;
    uint64_t pend = __ballot(counted);
    while (pend) {
      const int32_t gx = __builtin_amdgcn_readlane(g, __ffsll((unsigned long long)pend) - 1);
      const bool mine = counted && g == gx;
      pend &= ~__ballot(mine);
      const int64_t su = wave_sum64(mine ? ubv : 0), mx = wave_max64(mine ? f1 + fu : 0);
      if (lane() == 0) {
        atomicAdd((unsigned long long *)&gstat[gx * kStCount + kStUb], (unsigned long long)su);
        atomicMax((unsigned long long *)&gstat[gx * kStCount + kStMaxFlops], (unsigned long long)mx);
      }
    }
    append(valid && tier == 0, (int32_t)v, tiny, &counters[kCtTiny]);
    append(valid && tier == 1, (int32_t)v, mid, &counters[kCtMid]);
  }
}

// Groups whose count-pass multiplication totals a tiny-chain workgroup sums
// in LDS before its global atomics.
constexpr int kChainLdsGroups = 64;

// Tiny chain vector: one wavefront, both stages in registers.
template <int K, bool COUNT>
__device__ __forceinline__ void chain_tiny(const Plan &P, const ChainDev *chains, int64_t v, int64_t *gstat,
                                           unsigned long long *s_fl) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int l = lane();
  const int32_t p = uload(P.seg_prod + v), t = uload(P.seg_svec + v);
  const ChainDev C = uload(chains + p);
  // stage 1: one product of G1 (x) s per lane
  int key = INT32_MAX;
  T val = T();
  int filled = 0;
  const int64_t e1 = uload(C.s_ptr + t + 1);
  for (int64_t eb = uload(C.s_ptr + t); eb < e1; eb += kWave) {
    const int64_t e = eb + l;
    int len = 0;
    int64_t gb = 0;
    T sv = T();
    if (e < e1) {
      const int32_t q = gload(C.s_idx + e);
      if (q >= 0 && q < C.g1_nvec) {
        gb = gload(C.g1_ptr + q);
        len = (int)(gload(C.g1_ptr + q + 1) - gb);
        if (SR::kVal) sv = gload((const T *)C.s_val + e);
      }
    }
    const int Pp = wave_incl_scan(len);
    const int tot = read_lane(Pp, kWave - 1);
    if (tot == 0) continue;
    const int f = l - filled;
    const bool mine = f >= 0 && f < tot;
    const int o = owner_of(Pp, mine ? f : 0);
    const int64_t st = __shfl(gb - (int64_t)(Pp - len), o, kWave);
    const T so = __shfl(sv, o, kWave);
    if (mine) {
      key = gload(C.g1_idx + st + f);
      if (SR::kVal) val = SR::mul(so, gload((const T *)C.g1_val + st + f));
    }
    filled += tot;
  }
  const bool t1 = sort_merge64<SR>(key, val, C.t_minor < kPackMinor);
  // stage 2: every merged entry (k, t) of T streams G2(:, k)
  int len = 0;
  int64_t gb = 0;
  if (t1 && key < C.g2_nvec) {
    gb = gload(C.g2_ptr + key);
    len = (int)(gload(C.g2_ptr + key + 1) - gb);
  }
  const int Pp = wave_incl_scan(len);
  const int tot = read_lane(Pp, kWave - 1);
  const int o = owner_of(Pp, l < tot ? l : 0);
  const int64_t st = __shfl(gb - (int64_t)(Pp - len), o, kWave);
  const T so = SR::kVal ? __shfl(val, o, kWave) : T();
  int key2 = INT32_MAX;
  T val2 = T();
  if (l < tot) {
    key2 = gload(C.g2_idx + st + l);
    if (SR::kVal) val2 = SR::mul(so, gload((const T *)C.g2_val + st + l));
  }
  const bool tail = sort_merge64<SR>(key2, val2, uload(&P.groups[C.group].minor) < kPackMinor);
  const uint64_t hm = __ballot(tail);
  if (COUNT) {
    if (l == 0) {
      P.ov_cnt[v] = __popcll(hm);
      // the group's multiplications: into the workgroup's LDS total for the
      // first kChainLdsGroups groups (one global atomic per group and
      // workgroup at the end), straight to the global total beyond them
      const unsigned long long fl = (unsigned long long)(filled + tot);
      if (C.group < kChainLdsGroups) atomicAdd(&s_fl[C.group], fl);
      else atomicAdd((unsigned long long *)&gstat[C.group * kStCount + kStFlops], fl);
    }
    return;
  }
  chk_count(P, l == 0 && (int64_t)__popcll(hm) != gload(P.ov_cnt + v));
  if (tail) {
    const int r = __popcll(hm & ((1ull << l) - 1ull));
    const OutDev O = uload(P.outs + C.group);
    const int64_t pos = out_offset(P, v) + r;
    gstore(O.idx + pos, key2);
    if (SR::kVal) gstore((T *)O.val + pos, val2);
  }
}

// Open-addressing LDS hash insert (ids stored as id + 1, 0 = empty).
template <class SR, bool ACC>
__device__ __forceinline__ int hash_insert(uint32_t *keys, typename SR::Slot *vals, int logts, int id,
                                           typename SR::T x) {
  const uint32_t kk = (uint32_t)id + 1u;
  const int mask = (1 << logts) - 1;
  int h = (int)hash_id((uint32_t)id, logts);
  while (true) {
    uint32_t cur = keys[h];
    if (cur == 0) cur = atomicCAS(&keys[h], 0u, kk);
    if (cur == 0 || cur == kk) break;
    h = (h + 1) & mask;
  }
  if (ACC) SR::acc(&vals[h], x);
  return h;
}

// Mid chain vector: one workgroup. Stage 1 into hash 1 (ts slots), its
// entries compacted into T (ids, values), stage 2 into hash 2 (ts slots),
// sorted by id in LDS and written. LDS: 2 * ts keys, 2 * ts value slots and
// ts / 2 T entries; every word is zero again at the end.
template <int K, bool COUNT>
__device__ void chain_mid(const Plan &P, const ChainDev *chains, int64_t v, uint32_t *lds, int64_t *scratch, int ts,
                          int64_t *gstat) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  typedef typename SR::Slot Slot;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wid = tid / kWave, nw = nt / kWave;
  int logts = 0;
  while ((1 << logts) < ts) ++logts;
  uint32_t *k1 = lds;
  uint32_t *k2 = lds + ts;
  int32_t *tk = (int32_t *)(lds + 2 * ts);              // T ids (ts / 2)
  Slot *v1 = (Slot *)(lds + 2 * ts + ts / 2);           // aligned: ts is a power of two >= 64
  Slot *v2 = v1 + ts;
  Slot *tv = v2 + ts;                                   // T values (ts / 2)
  const int32_t p = uload(P.seg_prod + v), t = uload(P.seg_svec + v);
  const ChainDev C = uload(chains + p);
  // stage 1: waves take batches of 64 S entries; each entry's G1 vector flat over the lanes
  // (the count pass needs only the ids of T and of C: no values)
  auto ins1 = step<T>([&](int id, T x) { hash_insert<SR, !COUNT>(k1, v1, logts, id, x); });
  const int64_t e1 = uload(C.s_ptr + t + 1);
  int64_t f1 = 0;
  for (int64_t eb = uload(C.s_ptr + t) + (int64_t)wid * kWave; eb < e1; eb += (int64_t)nw * kWave) {
    const int64_t e = eb + lane();
    int len = 0;
    int64_t gb = 0;
    T sv = T();
    if (e < e1) {
      const int32_t q = gload(C.s_idx + e);
      if (q >= 0 && q < C.g1_nvec) {
        gb = gload(C.g1_ptr + q);
        len = (int)(gload(C.g1_ptr + q + 1) - gb);
        if (SR::kVal) sv = gload((const T *)C.s_val + e);
      }
    }
    f1 += len;
    run_batch<SR>(len, gb, sv, C.g1_idx, (const T *)C.g1_val, ins1);
  }
  __syncthreads();
  // T: the occupied slots of hash 1, compacted (order is irrelevant to stage 2)
  int local = 0;
  for (int i = tid; i < ts; i += nt) local += k1[i] != 0;
  int64_t ntot;
  int64_t pos = block_excl_scan(local, scratch, &ntot);
  for (int i = tid; i < ts; i += nt) {
    if (k1[i] != 0) {
      tk[pos] = (int32_t)(k1[i] - 1u);
      if (SR::kVal) tv[pos] = v1[i];
      ++pos;
    }
    k1[i] = 0;
    v1[i] = Slot();
  }
  __syncthreads();
  // stage 2: waves take batches of 64 T entries
  auto ins2 = step<T>([&](int id, T x) { hash_insert<SR, !COUNT>(k2, v2, logts, id, x); });
  const int nT = (int)ntot;
  int64_t f2 = 0;
  for (int b = wid * kWave; b < nT; b += nw * kWave) {
    const int x = b + lane();
    int len = 0;
    int64_t gb = 0;
    T sv = T();
    if (x < nT) {
      const int32_t k = tk[x];
      if (k < C.g2_nvec) {
        gb = gload(C.g2_ptr + k);
        len = (int)(gload(C.g2_ptr + k + 1) - gb);
      }
      if (SR::kVal) sv = SR::dec(tv[x]);
    }
    f2 += len;
    run_batch<SR>(len, gb, sv, C.g2_idx, (const T *)C.g2_val, ins2);
  }
  __syncthreads();
  for (int i = tid; i < ts / 2; i += nt) {
    tk[i] = 0;
    tv[i] = Slot();
  }
  if (COUNT) {
    int64_t cnt = 0;
    for (int i = tid; i < ts; i += nt) {
      cnt += k2[i] != 0;
      k2[i] = 0;
      v2[i] = Slot();
    }
    const int64_t total = block_sum(cnt, scratch);
    const int64_t fl = block_sum(f1 + f2, scratch);
    if (tid == 0) {
      P.ov_cnt[v] = total;
      atomicAdd((unsigned long long *)&gstat[C.group * kStCount + kStFlops], (unsigned long long)fl);
    }
    __syncthreads();
    return;
  }
  // sort hash 2 by id (empty slots last), then write the first cnt slots
  for (int i = tid; i < ts; i += nt)
    if (k2[i] == 0) k2[i] = 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= ts; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (ts >> 1); i += nt) {
        const int lo = ((i / j) * 2 * j) + (i % j);
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint32_t a = k2[lo], b = k2[hi];
        if ((a > b) == up) {
          k2[lo] = b;
          k2[hi] = a;
          if (SR::kVal) {
            const Slot tmp = v2[lo];
            v2[lo] = v2[hi];
            v2[hi] = tmp;
          }
        }
      }
      __syncthreads();
    }
  }
  const OutDev O = uload(P.outs + C.group);
  const int64_t base = out_offset(P, v);
  const int64_t cnt = gload(P.ov_cnt + v);
  if constexpr (SG_CHECK) {
    // exactly cnt keys: slot cnt - 1 holds one, slot cnt is empty (read before any slot is cleared)
    chk_count(P, tid == 0 && ((cnt > 0 && k2[cnt - 1] == 0xFFFFFFFFu) || (cnt < ts && k2[cnt] != 0xFFFFFFFFu)));
    __syncthreads();
  }
  for (int i = tid; i < ts; i += nt) {
    if (i < cnt) {
      gstore(O.idx + base + i, (int32_t)(k2[i] - 1u));
      if (SR::kVal) gstore((T *)O.val + base + i, SR::dec(v2[i]));
    }
    k2[i] = 0;
    v2[i] = Slot();
  }
  __syncthreads();
}

// Count and numeric launches: tiny vectors one wavefront each (grid-stride);
// mid vectors one workgroup each from a device queue.
template <int K, bool COUNT>
__global__ void __launch_bounds__(256) k_chain_tiny(Plan P, const ChainDev *chains, int64_t *gstat) {
  const int64_t n = P.counters[kCtTiny];
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  __shared__ unsigned long long s_fl[kChainLdsGroups];
  if (COUNT) {
    if (threadIdx.x < kChainLdsGroups) s_fl[threadIdx.x] = 0;
    __syncthreads();
  }
  for (int64_t i = wave; i < n; i += nwaves) chain_tiny<K, COUNT>(P, chains, uload(P.tiny_list + i), gstat, s_fl);
  if (COUNT) {
    __syncthreads();
    if (threadIdx.x < kChainLdsGroups && s_fl[threadIdx.x])
      atomicAdd((unsigned long long *)&gstat[threadIdx.x * kStCount + kStFlops], s_fl[threadIdx.x]);
  }
}

template <int K, bool COUNT>
__global__ void __launch_bounds__(kBlockMax, kWavesPerSimd) k_chain_mid(Plan P, const ChainDev *chains, int64_t *queue,
                                                                     int ts, int64_t *gstat) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t scratch[kMaxWaves + 1];
  __shared__ int64_t s_item;
  zero_lds(lds, P.lds_words);
  const int64_t n = P.counters[kCtMid];
  while (true) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long *)queue, 1ull);
    __syncthreads();
    const int64_t i = uni(s_item);
    __syncthreads();
    if (i >= n) break;
    chain_mid<K, COUNT>(P, chains, uload(P.mid_list + i), lds, scratch, ts, gstat);
    chk_lds_zero(P, lds);
  }
}

}  // namespace sg
