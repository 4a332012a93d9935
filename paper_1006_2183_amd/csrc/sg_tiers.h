// Numeric tiers of the flops-binned local product, each in a count variant
// (exact size of an output vector or window) and a numeric variant (writes
// the sorted ids and accumulated values):
//
//   tiny   output vectors with at most 64 multiplications: the products
//          are placed one per lane, sorted by id with a register bitonic
//          network, and equal ids are merged by a segmented reduction (the
//          multiway merge of Section 2.4, done on 64 lanes instead of a
//          heap); several small vectors share one wavefront pass, sorted by
//          (vector, id);
//   mid    one workgroup per vector whose size bound fits in LDS:
//          bitmap-rank accumulator (a bit per output id marks the pattern,
//          a prefix count per 32-bit word turns an id into its rank, so the
//          values are accumulated densely and emitted already sorted), or
//          an open-addressing LDS hash followed by an in-LDS bitonic sort;
//   heavy  a count pass marks the vector's whole id range in an LDS bitmap
//          and records the entries per split bucket (a fixed run of ids);
//          windows of consecutive buckets are then planned so that each
//          fits the LDS value capacity, and every window is one workgroup
//          item of the bitmap-rank accumulator restricted to its ids. Where
//          the id range is narrow enough for one dense window (or the
//          bitmap would not fit), a window is instead a dense LDS sparse
//          accumulator (the SPA of Section 3.3: a flag bit and a value per
//          id). The gathered operand is read in place through per-vector
//          split points at bucket boundaries.
//
// Every workgroup keeps its dynamic LDS at all-zero bits between items; the
// semiring traits encode the additive identity as zero bits.
#pragma once

#include "sg_device.h"

namespace sg {

// Invariant checks of the SG_CHECK build (no code in the normal build).
// chk_lds_zero: called by every thread of a persistent workgroup between two
// work items; counts the items after which the dynamic LDS is not all-zero.
__device__ __forceinline__ void chk_lds_zero(const Plan &P, const uint32_t *lds) {
  if constexpr (SG_CHECK) {
    int bad = 0;
    for (int i = threadIdx.x; i < P.lds_words; i += blockDim.x) bad |= lds[i] != 0u;
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicAdd((unsigned long long *)&P.chk[kCtChkLds], 1ull);
  }
}
// chk_count: counts a numeric result whose entry count differs from the plan.
__device__ __forceinline__ void chk_count(const Plan &P, bool bad) {
  if constexpr (SG_CHECK) {
    if (bad) atomicAdd((unsigned long long *)&P.chk[kCtChkCount], 1ull);
  }
}

// The output mask of vector v (its group's mask at v's major id).
struct MaskRef {
  const uint32_t *m;
  int64_t stride;
  int64_t j;
  int32_t comp;
  __device__ __forceinline__ bool on() const { return m != nullptr; }
  // bits of the ids [32 w, 32 w + 32) the output keeps
  __device__ __forceinline__ uint32_t word(int64_t w) const { return keep_word(m, stride, comp, j, w); }
  __device__ __forceinline__ bool keeps(int64_t id) const { return m == nullptr || ((word(id >> 5) >> (id & 31)) & 1u); }
};
__device__ __forceinline__ MaskRef mask_of(const Plan &P, int64_t v) {
  const int32_t g = uload(P.ov_group + v);
  MaskRef r{uload(&P.groups[g].mask), 0, 0, 0};
  if (r.m) {
    r.stride = uload(&P.groups[g].mask_stride);
    r.comp = uload(&P.groups[g].mask_comp);
    r.j = uload(P.ov_id + v);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Accumulators take a product in two steps so that the LDS reads of several
// products can be in flight together: prep(id) issues the reads one product
// needs and returns them as a token, commit(id, token, value) applies it.
// Step wraps a one-step lambda. kFlat picks the walk (flat over the lanes
// or lane groups per entry); kSpread has the flat walk hand neighbouring
// lanes products nine apart, which keeps bitmap-word atomics of one
// instruction off a common word; kRounds is the flat walk's rounds in
// flight (bitmap marks hold no values: eight fit the registers).
template <class T, class F, bool FLAT = false>
struct Step {
  static constexpr bool kFlat = FLAT;
  static constexpr bool kSpread = FLAT;
  static constexpr int kRounds = 8;
  F f;
  __device__ __forceinline__ uint64_t prep(int) const { return 0; }
  __device__ __forceinline__ void commit(int id, uint64_t, T v) { f(id, v); }
};
template <class T, class F>
__device__ __forceinline__ Step<T, F> step(F f) {
  return Step<T, F>{f};
}
template <class T, class F>
__device__ __forceinline__ Step<T, F, true> flat_step(F f) {
  return Step<T, F, true>{f};
}

// Products of one batch of (up to) 64 stored entries of S, one per lane: the
// lane holds `len` products in G positions [gb, gb + len) with S value sv.
// Every product is passed to the accumulator once.
//
// The wavefront splits into groups of gs lanes, gs the power of two nearest
// above the batch's mean length (1..64); the 64 / gs groups each take a
// different entry at a time and stride its G positions, so that short and
// long G vectors both keep every lane busy and the groups' loads are in
// flight together. Entries with products are compacted through a per-wave
// LDS byte map so that empty ones cost nothing.
__shared__ uint8_t s_own[kMaxWaves * kWave];

template <class SR, class Act>
__device__ __forceinline__ void run_batch(int len, int64_t gb, typename SR::T sv, const int32_t *__restrict__ gidx,
                                          const typename SR::T *__restrict__ gval, Act &act) {
  typedef typename SR::T T;
  const int l = lane();
  const uint64_t m = __ballot(len > 0);
  if (m == 0) return;
  const int nz = __popcll(m);
  const int tot = wave_sum(len);
  const int avg = (tot + nz - 1) / nz;
  int lg = 0;
  while (lg < 6 && (1 << lg) < avg) ++lg;
  const int gs = 1 << lg;
  const int ng = kWave >> lg;
  const int gi = l >> lg;
  // position of this lane inside its group's run of gs consecutive products:
  // a bijection that puts neighbouring lanes 9 products apart, so that the
  // sorted ids of neighbouring lanes seldom share a 32-id bitmap word (same
  // word atomics serialise in LDS); the run's cache lines are unchanged
  const int li = ((l & (gs - 1)) * 9) & (gs - 1);
  uint8_t *own = s_own + (threadIdx.x / kWave) * kWave;
  if (len > 0) own[__popcll(m & ((1ull << l) - 1ull))] = (uint8_t)l;
  __builtin_amdgcn_wave_barrier();
  const int rounds = (nz + ng - 1) / ng;
  // four rounds at a time: the first product of four entries per lane is
  // gathered before any is committed, so four loads are in flight per lane
  // even when every entry fits its lane group; longer entries finish in the
  // unrolled tail loop below
  for (int rd = 0; rd < rounds; rd += 4) {
    int L[4];
    int64_t b[4];
    T sv4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = (rd + k) * ng + gi;
      const bool valid = rd + k < rounds && r < nz;
      const int o = valid ? own[r] : 0;
      L[k] = __shfl(len, o, kWave);
      b[k] = __shfl(gb, o, kWave);
      sv4[k] = __shfl(sv, o, kWave);
      if (!valid) L[k] = 0;
    }
    int32_t i4[4];
    T v4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      i4[k] = 0;
      v4[k] = T();
      if (li < L[k]) {
        i4[k] = gload(gidx + b[k] + li);
        if (SR::kVal) v4[k] = gload(gval + b[k] + li);
      }
    }
    uint64_t t4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t4[k] = li < L[k] ? act.prep(i4[k]) : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (li < L[k]) act.commit(i4[k], t4[k], SR::kVal ? SR::mul(sv4[k], v4[k]) : T());
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int Lk = L[k];
      if (Lk <= gs) continue;
      const int64_t bk = b[k];
      const T s = sv4[k];
      int f = li + gs;
      for (; f + 3 * gs < Lk; f += 4 * gs) {
        const int64_t g0 = bk + f;
        const int32_t i0 = gload(gidx + g0), i1 = gload(gidx + g0 + gs);
        const int32_t i2 = gload(gidx + g0 + 2 * gs), i3 = gload(gidx + g0 + 3 * gs);
        T v0 = T(), v1 = T(), v2 = T(), v3 = T();
        if (SR::kVal) {
          v0 = gload(gval + g0);
          v1 = gload(gval + g0 + gs);
          v2 = gload(gval + g0 + 2 * gs);
          v3 = gload(gval + g0 + 3 * gs);
        }
        const uint64_t t0 = act.prep(i0), t1 = act.prep(i1), t2 = act.prep(i2), t3 = act.prep(i3);
        act.commit(i0, t0, SR::kVal ? SR::mul(s, v0) : T());
        act.commit(i1, t1, SR::kVal ? SR::mul(s, v1) : T());
        act.commit(i2, t2, SR::kVal ? SR::mul(s, v2) : T());
        act.commit(i3, t3, SR::kVal ? SR::mul(s, v3) : T());
      }
      for (; f < Lk; f += gs) {
        const int64_t g = bk + f;
        const int32_t i = gload(gidx + g);
        const T v = SR::kVal ? gload(gval + g) : T();
        act.commit(i, act.prep(i), SR::kVal ? SR::mul(s, v) : T());
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Products of one batch of (up to) 64 stored entries of S, one per lane
// (lane e holds `len` products at G positions [gb, gb + len) with S value
// sv), spread flat over the lanes: product f (in entry order) goes to lane
// f mod 64 of round f / 64 (with Act::kSpread, lane l takes product 9 l mod
// 64 of the round), so every round but the last keeps all 64 lanes busy
// whatever the entry lengths. R rounds at a time have all their gathers in
// flight before the accumulator sees any.
// The entry of a lane's product: a round inside one entry (the common case
// of long G vectors) reads that entry's G base and S value as scalars; a
// round where a few entries start takes them in order with one compare per
// lane each; otherwise a binary search of the lanes' inclusive product
// counts. Lanes past the last product load the last product again (always
// in range) and skip the accumulator.
// PTR: the entries come from several products, so each lane holds the
// addresses of its entry's first G id (gb) and first G value (gv) instead
// of a position in one product's arrays (gidx, gval unused).
template <class SR, class Act, bool PTR, int R = Act::kRounds>
__device__ __forceinline__ void flat_walk(int len, int64_t gb, int64_t gv, typename SR::T sv,
                                          const int32_t *__restrict__ gidx, const typename SR::T *__restrict__ gval,
                                          Act &act) {
  typedef typename SR::T T;
  constexpr int kFewStarts = 4;
  constexpr bool kTwo = PTR && SR::kVal;  // a second base per entry (its values)
  const int l = lane();
  const int pl = Act::kSpread ? ((l * 9) & (kWave - 1)) : l;  // this lane's product within a round
  const int incl = wave_incl_scan(len);
  const int tot = read_lane(incl, kWave - 1);
  if (tot == 0) return;
  const int st = incl - len;
  // product f of this entry: G position gbase + f, or (PTR) id at address
  // gbase + 4 f and value at vbase + sizeof(T) f
  const int64_t gbase = PTR ? gb - (int64_t)st * (int64_t)sizeof(int32_t) : gb - st;
  const int64_t vbase = kTwo ? gv - (int64_t)st * (int64_t)sizeof(T) : 0;
  const bool live = len > 0;
  for (int j0 = 0; j0 < tot; j0 += R * kWave) {
    int64_t g[R];
    int64_t gw[kTwo ? R : 1];  // value addresses (PTR with values only)
    T s4[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int f0 = j0 + k * kWave;
      const int r0 = f0 < tot ? f0 : tot - 1;          // first product of the round, clamped
      const int fl = f0 + pl < tot ? f0 + pl : tot - 1;  // this lane's product, clamped
      const int e0 = (int)__popcll(__ballot(incl <= r0));                // entry of product r0
      const uint64_t starts = __ballot(live && st > r0 && st < f0 + kWave);  // entries starting later in the round
      // G position (or id address) of this lane's product, from its entry's base
      constexpr int64_t kStep = PTR ? (int64_t)sizeof(int32_t) : 1;
      if (starts == 0) {
        g[k] = read_lane64(gbase, e0) + (int64_t)fl * kStep;
        if constexpr (kTwo) gw[k] = read_lane64(vbase, e0) + (int64_t)fl * (int64_t)sizeof(T);
        if constexpr (SR::kVal) s4[k] = read_lane_val(sv, e0);
        else s4[k] = T();
      } else {
        int e = e0;
        if (__popcll(starts) <= kFewStarts) {
          uint64_t m = starts;
          while (m) {
            const int x = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            if (fl >= read_lane(st, x)) e = x;
          }
        } else {
          e = owner_of(incl, fl);
        }
        g[k] = __shfl(gbase, e, kWave) + (int64_t)fl * kStep;
        if constexpr (kTwo) gw[k] = __shfl(vbase, e, kWave) + (int64_t)fl * (int64_t)sizeof(T);
        s4[k] = __shfl(sv, e, kWave);
      }
    }
    int32_t i4[R];
    T v4[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if constexpr (PTR) {
        i4[k] = gload((const int32_t *)g[k]);
        if constexpr (kTwo) v4[k] = gload((const T *)gw[k]);
        else v4[k] = T();
      } else {
        i4[k] = gload(gidx + g[k]);
        v4[k] = SR::kVal ? gload(gval + g[k]) : T();
      }
    }
    uint64_t t4[R];
    if (j0 + R * kWave <= tot) {  // every lane's products are real: no masks
#pragma unroll
      for (int k = 0; k < R; ++k) t4[k] = act.prep(i4[k]);
#pragma unroll
      for (int k = 0; k < R; ++k) act.commit(i4[k], t4[k], SR::kVal ? SR::mul(s4[k], v4[k]) : T());
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) t4[k] = j0 + k * kWave + pl < tot ? act.prep(i4[k]) : 0;
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (j0 + k * kWave + pl < tot) act.commit(i4[k], t4[k], SR::kVal ? SR::mul(s4[k], v4[k]) : T());
    }
  }
  __builtin_amdgcn_wave_barrier();
}

template <class SR, class Act>
__device__ __forceinline__ void run_flat(int len, int64_t gb, typename SR::T sv, const int32_t *__restrict__ gidx,
                                         const typename SR::T *__restrict__ gval, Act &act) {
  flat_walk<SR, Act, false>(len, gb, 0, sv, gidx, gval, act);
}

// Load the lane's stored S entry e of product d and describe its products:
// the whole G vector (b0 < 0) or only its ids in split buckets [b0, b1).
template <class SR>
__device__ __forceinline__ void load_entry(const ProdDev &d, int64_t e, int64_t e1, int b0, int b1, int &len,
                                           int64_t &gb, typename SR::T &sv) {
  typedef typename SR::T T;
  len = 0;
  gb = 0;
  sv = T();
  if (e >= e1) return;
  const int32_t k = gload(d.s_idx + e);
  const int32_t gt = d.gres ? gload(d.gres + e) : ((k >= 0 && k < d.g_nvec) ? k : -1);
  if (gt < 0) return;
  const int64_t p0 = gload(d.g_ptr + gt);
  if (b0 >= 0 && d.wsplit) {
    const int32_t *ws = d.wsplit + (int64_t)gt * (d.nsplit + 1);
    const int32_t w0 = gload(ws + b0);
    gb = p0 + w0;
    len = gload(ws + b1) - w0;
  } else {
    gb = p0;
    len = (int)(gload(d.g_ptr + gt + 1) - p0);
  }
  if (SR::kVal) sv = gload((const T *)d.s_val + e);
}

// All products of output vector v (restricted to split buckets [b0, b1) if
// b0 >= 0), shared by the nw wavefronts of the caller. With fewer segments
// than wavefronts, every wave walks the same batches of 64 stored S
// entries; the products of a batch, in entry order, are cut into nw equal
// slices and wave wid takes slice wid by clipping each entry's G range to
// it. A vector with few entries but long G vectors (the typical heavy
// vector) thus keeps every wave busy.
template <class SR, class Act>
__device__ __forceinline__ void for_products(const Plan &P, int64_t v, int b0, int b1, int wid, int nw, Act &act) {
  typedef typename SR::T T;
  const int64_t s0 = uload(P.ov_seg + v), s1 = uload(P.ov_seg + v + 1);
  // many segments (stage products accumulated into one vector): the
  // segments are dealt to the wavefronts round robin and each wavefront
  // takes every product of its own segments (one slice), so no wavefront
  // walks the descriptors of all of them
  const bool many = s1 - s0 >= nw;
  const int uw = uni(wid);  // the wavefront index is wave-uniform: keep the walk scalar
  const int sid = many ? 0 : uw, sn = many ? 1 : nw;
  for (int64_t s = s0 + (many ? uw : 0); s < s1; s += many ? nw : 1) {
    const ProdDev d = uload(P.prods + uload(P.seg_prod + s));
    const int32_t t = uload(P.seg_svec + s);
    const int64_t e1 = uload(d.s_ptr + t + 1);
    for (int64_t eb = uload(d.s_ptr + t); eb < e1; eb += kWave) {
      int len;
      int64_t gb;
      T sv;
      load_entry<SR>(d, eb + lane(), e1, b0, b1, len, gb, sv);
      const int incl = wave_incl_scan(len);
      const int tot = read_lane(incl, kWave - 1);
      if (tot == 0) continue;
      const int f0 = (int)((int64_t)tot * sid / sn);
      const int f1 = (int)((int64_t)tot * (sid + 1) / sn);
      const int st = incl - len;
      const int a = st > f0 ? st : f0;
      const int e = incl < f1 ? incl : f1;
      const int len2 = e > a ? e - a : 0;
      // the rank accumulator (numeric windows) takes the products flat over
      // the lanes; bitmap marks and dense windows keep the entry groups,
      // whose lane layout suits their LDS atomics better
      if constexpr (Act::kFlat)
        run_flat<SR>(len2, gb + (a - st), sv, d.g_idx, (const T *)d.g_val, act);
      else
        run_batch<SR>(len2, gb + (a - st), sv, d.g_idx, (const T *)d.g_val, act);
    }
  }
}

// All products of a heavy window from its entry records [rb, rb + nrec):
// one load level per batch of 64 entries (the addresses of the entry's G
// slice inside the window and its S value) instead of the segment's
// descriptors, the entry, its G vector and its window split points in turn.
// Records name addresses, so a vector fed by several products (a SUMMA
// share's stage products) walks them as one list. With at least as many
// batches as wavefronts, the batches are dealt to the wavefronts round robin
// and each takes all products of its own batches, so the chains of record
// and gather loads run side by side instead of one batch after another;
// with fewer (but more than one), each batch is shared by the wavefronts
// whose index it is modulo the batch count; with one, every wavefront takes
// its slice of it.
template <class SR, class Act>
__device__ __forceinline__ void for_products_recs(const Plan &P, int64_t rb, int32_t nrec, int wid, int nw,
                                                  Act &act) {
  typedef typename SR::T T;
  static_assert(Act::kFlat, "records feed the flat walk");
  const int uw = uni(wid);
  const int64_t nbatch = ((int64_t)nrec + kWave - 1) / kWave;
  const bool many = nbatch >= nw;
  if (!many && nbatch > 1) {
    // fewer batches than wavefronts: each wavefront takes one batch (b =
    // its index mod nbatch) and its slice of that batch's products, so every
    // wavefront reads one level of records instead of one per batch
    const int b = uw % (int)nbatch;
    const int sid = uw / (int)nbatch, sn = (nw - b + (int)nbatch - 1) / (int)nbatch;
    const int64_t x = rb + (int64_t)b * kWave + lane();
    const bool ok = (int64_t)b * kWave + lane() < nrec;
    const int len = ok ? gload(P.rec_len + x) : 0;
    const int64_t gi = ok ? gload(P.rec_gi + x) : 0;
    const int64_t gv = (SR::kVal && ok) ? gload(P.rec_gv + x) : 0;
    const T sv = (SR::kVal && ok) ? gload((const T *)P.rec_sv + x) : T();
    const int incl = wave_incl_scan(len);
    const int tot = read_lane(incl, kWave - 1);
    if (tot == 0) return;
    const int f0 = (int)((int64_t)tot * sid / sn);
    const int f1 = (int)((int64_t)tot * (sid + 1) / sn);
    const int st = incl - len;
    const int a = st > f0 ? st : f0;
    const int e = incl < f1 ? incl : f1;
    const int len2 = e > a ? e - a : 0;
    const int64_t skip = a > st ? a - st : 0;
    flat_walk<SR, Act, true>(len2, gi + skip * (int64_t)sizeof(int32_t), gv + skip * (int64_t)sizeof(T), sv, nullptr,
                             nullptr, act);
    return;
  }
  const int sid = many ? 0 : uw, sn = many ? 1 : nw;
  const int64_t step = (many ? nw : 1) * (int64_t)kWave;
  // the next batch's records are requested before this batch's gathers, so
  // the two load levels of consecutive batches overlap
  int64_t eb = (many ? uw : 0) * (int64_t)kWave;
  int len_n = 0;
  int64_t gi_n = 0, gv_n = 0;
  T sv_n = T();
  auto fetch = [&](int64_t b) {
    const int64_t x = rb + b + lane();
    const bool ok = b + lane() < nrec;
    len_n = ok ? gload(P.rec_len + x) : 0;
    gi_n = ok ? gload(P.rec_gi + x) : 0;
    gv_n = (SR::kVal && ok) ? gload(P.rec_gv + x) : 0;
    sv_n = (SR::kVal && ok) ? gload((const T *)P.rec_sv + x) : T();
  };
  if (eb < nrec) fetch(eb);
  for (; eb < nrec; eb += step) {
    const int len = len_n;
    const int64_t gi = gi_n, gv = gv_n;
    const T sv = sv_n;
    if (eb + step < nrec) fetch(eb + step);
    const int incl = wave_incl_scan(len);
    const int tot = read_lane(incl, kWave - 1);
    if (tot == 0) continue;
    const int f0 = (int)((int64_t)tot * sid / sn);
    const int f1 = (int)((int64_t)tot * (sid + 1) / sn);
    const int st = incl - len;
    const int a = st > f0 ? st : f0;
    const int e = incl < f1 ? incl : f1;
    const int len2 = e > a ? e - a : 0;
    const int64_t skip = a > st ? a - st : 0;  // products of the entry before this wave's slice
    flat_walk<SR, Act, true>(len2, gi + skip * (int64_t)sizeof(int32_t), gv + skip * (int64_t)sizeof(T), sv, nullptr,
                             nullptr, act);
  }
}

__device__ __forceinline__ int64_t out_offset(const Plan &P, int64_t v) {
  return uload(P.ov_off + v) - uload(&P.groups[uload(P.ov_group + v)].nnz_base);
}

// ---------------------------------------------------------------------------
// Ids below kPackMinor - 1 pack with their 6-bit lane into one 32-bit key.
constexpr int64_t kPackMinor = (int64_t)1 << 26;

// Ascending bitonic sort of one 32-bit key per lane across the 64 lanes: a
// lane exchange, a min, a max and a select per step.
__device__ __forceinline__ void bitonic64_u32(uint32_t &kp) {
  const int l = lane();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t pk = xor_lane(kp, j);
      const uint32_t mn = pk < kp ? pk : kp, mx = pk < kp ? kp : pk;
      kp = ((l & k) == 0) == ((l & j) == 0) ? mn : mx;
    }
  }
}

// Bitonic sort of (key, val) across the 64 lanes by key (INT32_MAX: empty
// lane), then the segmented (+) of equal keys: the last lane of each run
// holds the run's total, and the result says whether this lane is such a
// last lane. With `pack` (every id of the vector's range below kPackMinor -
// 1) only the 32-bit key id << 6 | lane moves through the network, as a min,
// a max and a select per step, and each lane then reads its value from the
// lane its key names; equal ids end up in lane order. Otherwise key and
// value move together, by two selects per step. The tiny tiers spend most of
// their instructions here, and the packed form takes about a third of them.
template <class SR>
__device__ __forceinline__ bool sort_merge64(int &key, typename SR::T &val, bool pack) {
  typedef typename SR::T T;
  const int l = lane();
  if (pack) {
    uint32_t kp = key == INT32_MAX ? 0xFFFFFFFFu : ((uint32_t)key << 6) | (uint32_t)l;
    bitonic64_u32(kp);
    if (SR::kVal) val = __shfl(val, (int)(kp & (uint32_t)(kWave - 1)), kWave);
    key = kp == 0xFFFFFFFFu ? INT32_MAX : (int)(kp >> 6);
  } else {
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int pk = xor_lane(key, j);
        const T pv = SR::kVal ? xor_lane(val, j) : T();
        cmp_exchange(key, val, pk, pv, ((l & k) == 0) == ((l & j) == 0));
      }
    }
  }
  const uint64_t k64 = (uint64_t)(uint32_t)key;
  if (SR::kVal) val = seg_prefix<SR>(k64, val);
  return key != INT32_MAX && next_lane_key(k64) != k64;
}

// Tiny tier: one wavefront, at most 64 products.
template <int K, bool COUNT>
__device__ __forceinline__ void tiny_vector(const Plan &P, int64_t v) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int l = lane();
  int key = INT32_MAX;
  T val = T();
  int filled = 0;
  const int64_t s0 = uload(P.ov_seg + v), s1 = uload(P.ov_seg + v + 1);
  for (int64_t s = s0; s < s1; ++s) {
    const ProdDev d = uload(P.prods + uload(P.seg_prod + s));
    const int32_t t = uload(P.seg_svec + s);
    const int64_t e1 = uload(d.s_ptr + t + 1);
    for (int64_t eb = uload(d.s_ptr + t); eb < e1; eb += kWave) {
      int len;
      int64_t gb;
      T sv;
      load_entry<SR>(d, eb + l, e1, -1, -1, len, gb, sv);
      const int Pp = wave_incl_scan(len);
      const int tot = read_lane(Pp, kWave - 1);
      if (tot == 0) continue;
      const int f = l - filled;
      const bool mine = f >= 0 && f < tot;
      const int o = owner_of(Pp, mine ? f : 0);
      const int64_t start = gb - (int64_t)(Pp - len);
      const int64_t st = __shfl(start, o, kWave);
      const T so = __shfl(sv, o, kWave);
      if (mine) {
        const int64_t g = st + f;
        key = gload(d.g_idx + g);
        if (SR::kVal) val = SR::mul(so, gload((const T *)d.g_val + g));
      }
      filled += tot;
    }
  }
  // sort by id and (+) of equal ids: the last lane of each run ends with its total
  const int64_t minor = uload(&P.groups[uload(P.ov_group + v)].minor);
  bool tail = sort_merge64<SR>(key, val, minor < kPackMinor);
  const MaskRef mk = mask_of(P, v);
  if (mk.on() && tail) tail = mk.keeps(key);
  const uint64_t hm = __ballot(tail);
  if (COUNT) {
    if (l == 0) P.ov_cnt[v] = __popcll(hm);
    return;
  }
  chk_count(P, l == 0 && (int64_t)__popcll(hm) != gload(P.ov_cnt + v));
  if (tail) {
    const int r = __popcll(hm & ((1ull << l) - 1ull));
    const OutDev O = uload(P.outs + uload(P.ov_group + v));
    const int64_t pos = out_offset(P, v) + r;
    gstore(O.idx + pos, key);
    if (SR::kVal) gstore((T *)O.val + pos, val);
  }
}

// Tiny tier, packed: one wavefront takes tiny-list positions [c0, c1) (at
// most 64 vectors). Vectors with a single segment of the chunk's first
// product whose streamed entries fit the wave are packed: each round takes
// consecutive such vectors while their multiplications and their streamed
// entries each fit 64 lanes, places one streamed entry per lane, then one
// product per lane tagged with its vector's lane, sorts the 64 lanes by
// (vector, id), merges equal keys and writes each vector's run at its own
// offset. A vector with 7 multiplications thus costs a ninth of a
// wavefront pass instead of a whole one. The remaining vectors (several
// segments, another product, more than 64 streamed entries) take the
// one-vector path above.
__device__ __forceinline__ uint64_t lane_range(int a, int b) {
  const uint64_t hi = b >= kWave ? ~0ull : ((1ull << b) - 1ull);
  const uint64_t lo = a >= kWave ? ~0ull : ((1ull << a) - 1ull);
  return hi & ~lo;
}

// Tiny-list positions per wavefront chunk: enough chunks for every one of
// `waves` wavefronts, each at most 64 positions.
__device__ __forceinline__ int64_t tiny_chunk(int64_t n, int64_t waves) {
  const int64_t c = (n + waves - 1) / waves;
  return c < 1 ? 1 : (c > kWave ? kWave : c);
}

template <int K, bool COUNT>
__device__ __forceinline__ void tiny_pack(const Plan &P, int64_t c0, int64_t c1) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int l = lane();
  const bool has = c0 + l < c1;
  int64_t v = -1;
  int32_t p = -1, t = 0;
  int f = 0;
  int32_t jv = 0;  // the vector's output major id (for masked groups)
  if (has) {
    v = gload(P.tiny_list + c0 + l);
    jv = gload(P.ov_id + v);
    const int64_t s0 = gload(P.ov_seg + v), s1 = gload(P.ov_seg + v + 1);
    f = (int)gload(P.ov_flops + v);
    if (s1 - s0 == 1) {
      p = gload(P.seg_prod + s0);
      t = gload(P.seg_svec + s0);
    }
  }
  const uint64_t hasp = __ballot(p >= 0);
  bool pack = false;
  int64_t e0 = 0;
  int ne = 0;
  if (hasp) {
    const int32_t p0 = __builtin_amdgcn_readlane(p, __ffsll((unsigned long long)hasp) - 1);
    const ProdDev d = uload(P.prods + p0);
    if (p == p0) {
      e0 = gload(d.s_ptr + t);
      ne = (int)(gload(d.s_ptr + t + 1) - e0);
      pack = ne <= kWave && f <= kWave;
    }
    const int fp = pack ? f : 0, np = pack ? ne : 0;
    const int Finc = wave_incl_scan(fp), Einc = wave_incl_scan(np);
    const OutDev O = uload(P.outs + d.group);
    // (vector, id, lane) in one 32-bit sort key: 6 + 20 + 6 bits
    const bool pack32 = uload(&P.groups[d.group].minor) < ((int64_t)1 << 20);
    const uint32_t *gmask = uload(&P.groups[d.group].mask);
    int64_t gstride = 0;
    int32_t gcomp = 0;
    if (gmask) {
      gstride = uload(&P.groups[d.group].mask_stride);
      gcomp = uload(&P.groups[d.group].mask_comp);
    }
    int64_t opos = 0;
    if (!COUNT && pack) opos = gload(P.ov_off + v) - uload(&P.groups[d.group].nnz_base);
    uint64_t rem = __ballot(pack);
    while (rem) {
      const int first = __ffsll((unsigned long long)rem) - 1;
      const int bf = __builtin_amdgcn_readlane(Finc - fp, first);
      const int be = __builtin_amdgcn_readlane(Einc - np, first);
      const uint64_t sel = __ballot(((rem >> l) & 1ull) && Finc - bf <= kWave && Einc - be <= kWave);
      rem &= ~sel;
      const int last = 63 - __clzll((long long)sel);
      const int etot = __builtin_amdgcn_readlane(Einc, last) - be;
      const int ftot = __builtin_amdgcn_readlane(Finc, last) - bf;
      // one streamed entry per lane; j = the lane of its vector
      const bool ent = l < etot;
      const int j = owner_of(Einc - be, ent ? l : 0);
      const int64_t ej = __shfl(e0, j, kWave) + (l - (__shfl(Einc - np, j, kWave) - be));
      int len;
      int64_t gb;
      T sv;
      load_entry<SR>(d, ej, ent ? ej + 1 : ej, -1, -1, len, gb, sv);
      // one product per lane
      const int Pinc = wave_incl_scan(len);
      const int o = owner_of(Pinc, l < ftot ? l : 0);
      const int64_t st = __shfl(gb - (int64_t)(Pinc - len), o, kWave);
      const T so = __shfl(sv, o, kWave);
      const int tag_o = __shfl(j, o, kWave);
      uint64_t ck = ((uint64_t)kWave << 32) | 0x7fffffffull;
      T val = T();
      if (l < ftot) {
        const int64_t g = st + l;
        ck = ((uint64_t)tag_o << 32) | (uint32_t)gload(d.g_idx + g);
        if (SR::kVal) val = SR::mul(so, gload((const T *)d.g_val + g));
      }
      // bitonic sort of (vector, id) across the 64 lanes: packed keys with
      // each lane's value read back from the lane its key names, or key and
      // value moved together
      if (pack32) {
        uint32_t kp = l < ftot ? ((uint32_t)tag_o << 26) | ((uint32_t)ck << 6) | (uint32_t)l : 0xFFFFFFFFu;
        bitonic64_u32(kp);
        if (SR::kVal) val = __shfl(val, (int)(kp & (uint32_t)(kWave - 1)), kWave);
        ck = kp == 0xFFFFFFFFu ? (((uint64_t)kWave << 32) | 0x7fffffffull)
                               : (((uint64_t)(kp >> 26) << 32) | ((kp >> 6) & 0xFFFFFu));
      } else {
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
          for (int jj = k >> 1; jj > 0; jj >>= 1) {
            const uint64_t pk = xor_lane(ck, jj);
            const T pv = SR::kVal ? xor_lane(val, jj) : T();
            cmp_exchange(ck, val, pk, pv, ((l & k) == 0) == ((l & jj) == 0));
          }
        }
      }
      // segmented (+) of equal keys: the last lane of each run holds its total
      if (SR::kVal) val = seg_prefix<SR>(ck, val);
      const int tag = (int)(ck >> 32);
      bool tail = tag < kWave && next_lane_key(ck) != ck;
      if (gmask) {
        const int64_t jt = __shfl(jv, tag < kWave ? tag : 0, kWave);
        const uint32_t id = (uint32_t)ck;
        if (tail) tail = (keep_word(gmask, gstride, gcomp, jt, id >> 5) >> (id & 31)) & 1u;
      }
      const uint64_t hm = __ballot(tail);
      // vector lane x owns the sorted lanes [Finc_x - f_x - bf, Finc_x - bf)
      const int seg_a = Finc - fp - bf;
      if (COUNT) {
        if ((sel >> l) & 1ull) gstore(P.ov_cnt + v, (int64_t)__popcll(hm & lane_range(seg_a, Finc - bf)));
      } else {
        chk_count(P, ((sel >> l) & 1ull) &&
                         (int64_t)__popcll(hm & lane_range(seg_a, Finc - bf)) != gload(P.ov_cnt + v));
        const int src = tag < kWave ? tag : 0;
        const int a = __shfl(seg_a, src, kWave);
        const int64_t base = __shfl(opos, src, kWave);
        if (tail) {
          const int64_t pos = base + __popcll(hm & lane_range(a, l));
          gstore(O.idx + pos, (int32_t)(uint32_t)ck);
          if (SR::kVal) gstore((T *)O.val + pos, val);
        }
      }
    }
  }
  uint64_t fb = __ballot(has && !pack);
  while (fb) {
    const int x = __ffsll((unsigned long long)fb) - 1;
    fb &= fb - 1ull;
    const int64_t vx = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)((uint64_t)v >> 32), x) << 32) |
                                 (uint32_t)__builtin_amdgcn_readlane((int32_t)v, x));
    tiny_vector<K, COUNT>(P, vx);
  }
}

// ---------------------------------------------------------------------------
// LDS layout helpers (offsets in 32-bit words).
__device__ __forceinline__ int64_t align2(int64_t w) { return (w + 1) & ~(int64_t)1; }

// Bitmap-rank accumulator over output ids [lo, hi) of vector v: a bit per
// id marks the pattern, a prefix count per 32-bit word of bits turns an id
// into its rank, and the values are accumulated densely by rank, so the
// entries come out sorted without a sort. With values, each 32 ids own one
// 8-byte LDS word {bits, prefix}, so a rank costs one LDS read. b0 < 0 means
// the whole range (mid tier); else only the products in split buckets
// [b0, b1) are taken. COUNT writes the number of entries to ov_cnt[v]; the
// numeric variant writes them at out_pos.
// MASKED: the output mask removed ids from the bitmap, so products of those
// ids are skipped (a separate instantiation: the unmasked walk keeps no test
// in its innermost loop).
template <class SR, bool MASKED = false>
struct RankAcc {
  typedef typename SR::T T;
  typedef typename SR::Slot Slot;
  static constexpr bool kFlat = true;
  static constexpr bool kSpread = false;  // consecutive ranks: consecutive banks
  static constexpr int kRounds = 5;       // 4: 1% slower; 8: slower, more misses in flight only wait longer
  uint32_t *words;  // 2 x uint32 per 32 ids: bits, prefix
  Slot *vals;
  int lo32;
  __device__ __forceinline__ uint64_t prep(int id) const {
    const uint32_t r = (uint32_t)(id - lo32);
    return *(const uint64_t *)((const char *)words + ((r >> 2) & ~7u));  // the pair of word r / 32
  }
  __device__ __forceinline__ void commit(int id, uint64_t tok, T x) {
    const uint32_t r = (uint32_t)(id - lo32);
    const uint32_t bits = (uint32_t)tok;
    const uint32_t pre = (uint32_t)(tok >> 32);
    if (MASKED && !((bits >> (r & 31)) & 1u)) return;
    // set bits of the word below bit r % 32 (the field width is taken mod 32)
    SR::acc(&vals[pre + __popc(__builtin_amdgcn_ubfe(bits, 0u, r))], x);
  }
};

// Kept bitmap words [0, nwds) of a window (src) into the rank accumulator.
// The window is covered in passes of nt * kStage words; in a pass, thread t
// owns `per` consecutive words (per a multiple of 4, at most kStage) and
// stages them in registers, so all of its loads are in flight before the
// first wait; popcounts, a block scan and the writes follow from registers.
// With values (WS == 2) each word is written with its prefix (the count of
// set bits before it in the window). Pattern only (out_idx set), the ids are
// the result and are written straight to out_idx[rank]. Returns the count.
template <int WS>
__device__ __forceinline__ int64_t rank_load_kept(const uint32_t *src, int nwds, uint32_t *words, int64_t *scratch,
                                                  int32_t *out_idx = nullptr, int lo32 = 0) {
  constexpr int kStage = 16;
  const int tid = threadIdx.x, nt = blockDim.x;
  const bool vec = (((uintptr_t)src) & 15) == 0;
  int64_t run_total = 0;
  for (int base = 0; base < nwds; base += nt * kStage) {
    const int rem = nwds - base;
    int per = (rem + nt - 1) / nt;
    per = (per + 3) & ~3;
    if (per > kStage) per = kStage;
    const int w0 = base + tid * per;
    uint32_t r[kStage];
#pragma unroll
    for (int j = 0; j < kStage; j += 4) {
      const int w = w0 + j;
      if (j < per && w + 3 < nwds && vec) {
        const u32x4 x = gload((const u32x4 *)(src + w));
        r[j] = x.x;
        r[j + 1] = x.y;
        r[j + 2] = x.z;
        r[j + 3] = x.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) r[j + k] = (j + k < per && w + k < nwds) ? gload(src + w + k) : 0u;
      }
    }
    int local = 0;
#pragma unroll
    for (int j = 0; j < kStage; ++j) local += __popc(r[j]);
    int64_t total;
    int64_t run = block_excl_scan(local, scratch, &total) + run_total;
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int w = w0 + j;
      if (j < per && w < nwds) {
        if (out_idx) {
          uint32_t b = r[j];
          while (b) {
            const int bit = __ffs(b) - 1;
            b &= b - 1;
            gstore(out_idx + run, lo32 + (w << 5) + bit);
            ++run;
          }
        } else if (WS == 2) {
          *(uint2 *)&words[2 * w] = make_uint2(r[j], (uint32_t)run);
          run += __popc(r[j]);
        } else {
          words[w] = r[j];
          run += __popc(r[j]);
        }
      }
    }
    run_total += total;
  }
  return run_total;
}

template <int K, bool COUNT, bool WHOLE = false, bool RECS = false>
__device__ __forceinline__ int64_t rank_window(const Plan &P, int64_t v, int64_t lo, int64_t hi, int b0, int b1, int64_t out_pos,
                            uint32_t *lds, int64_t *scratch, const uint32_t *kept = nullptr, int64_t rb = -1,
                            int32_t nrec = 0) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  typedef typename SR::Slot Slot;
  // 32-bit LDS words per 32 ids: {bits, prefix} with values, bits alone
  // when counting or without values
  constexpr int WS = (SR::kVal && !COUNT) ? 2 : 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wid = tid / kWave, nw = nt / kWave;
  const int nwds = (int)((hi - lo + 31) >> 5);
  const int lo32 = (int)lo;
  uint32_t *words = lds;
  // a whole-range window (the mid tier) is mostly empty words: a second
  // bitmap with one bit per word of ids (top) lets the scan, the prefix
  // and the emit visit only the touched words
  constexpr bool two = WHOLE;  // whole id range, marked here (the mid tier)
  const int ntop = (nwds + 31) >> 5;
  uint32_t *top = lds + WS * nwds;
  Slot *vals = (Slot *)(lds + (two ? ((WS * nwds + ntop + 1) & ~1) : WS * nwds));
  const int tper = (ntop + nt - 1) / nt;  // top words per thread (contiguous)
  const int tw0 = tid * tper < ntop ? tid * tper : ntop;
  const int tw1 = tw0 + tper < ntop ? tw0 + tper : ntop;
  const OutDev O = uload(P.outs + uload(P.ov_group + v));
  const MaskRef mk = mask_of(P, v);
  const int64_t w0lo = lo >> 5;  // mask word of the window's first 32 ids
  int64_t cnt = 0;  // entries of the window

  if (!COUNT && kept) {
    // the count pass kept this vector's bitmap: the window's words arrive
    // with their prefixes, without a marking pass; pattern only, the kept
    // bits are the result
    if (!SR::kVal) {
      const int64_t n = rank_load_kept<WS>(kept + (lo >> 5), nwds, words, scratch, O.idx + out_pos, lo32);
      __syncthreads();
      return n;
    }
    cnt = rank_load_kept<WS>(kept + (lo >> 5), nwds, words, scratch);
    __syncthreads();
  } else if constexpr (two) {
    auto mark = flat_step<T>([&](int id, T) {
      const int r = id - lo32;
      const int w = r >> 5;
      atomicOr(&words[WS * w], 1u << (r & 31));
      atomicOr(&top[w >> 5], 1u << (w & 31));
    });
    if (RECS && rb >= 0) for_products_recs<SR>(P, rb, nrec, wid, nw, mark);
    else for_products<SR>(P, v, b0, b1, wid, nw, mark);
    __syncthreads();
    int local = 0;
    for (int tw = tw0; tw < tw1; ++tw) {
      uint32_t tb = top[tw];
      while (tb) {
        const int w = (tw << 5) + __ffs(tb) - 1;
        tb &= tb - 1;
        if (mk.on()) words[WS * w] &= mk.word(w0lo + w);  // drop the ids the output mask excludes
        local += __popc(words[WS * w]);
      }
    }
    int64_t total;
    const int64_t excl = block_excl_scan(local, scratch, &total);
    int64_t run = excl;
    for (int tw = tw0; tw < tw1; ++tw) {
      uint32_t tb = top[tw];
      while (tb) {
        const int w = (tw << 5) + __ffs(tb) - 1;
        tb &= tb - 1;
        const uint32_t b = words[WS * w];
        if (COUNT) {
          words[WS * w] = 0;
        } else if (!SR::kVal) {
          uint32_t bb = b;
          while (bb) {
            const int bit = __ffs(bb) - 1;
            bb &= bb - 1;
            gstore(O.idx + out_pos + run, lo32 + (w << 5) + bit);
            ++run;
          }
          words[w] = 0;
        } else {
          words[WS * w + 1] = (uint32_t)run;
          run += __popc(b);
        }
      }
      if (COUNT || !SR::kVal) top[tw] = 0;
    }
    if (COUNT) {
      if (tid == 0) gstore(P.ov_cnt + v, total);
      __syncthreads();
      return total;
    }
    if (!SR::kVal) {
      __syncthreads();
      return total;
    }
    cnt = total;
    __syncthreads();
  } else {
    auto mark = flat_step<T>([&](int id, T) {
      const int r = id - lo32;
      atomicOr(&words[WS * (r >> 5)], 1u << (r & 31));
    });
    for_products<SR>(P, v, b0, b1, wid, nw, mark);
    __syncthreads();

    // per-thread contiguous word range
    const int per = (nwds + nt - 1) / nt;
    const int w0 = tid * per < nwds ? tid * per : nwds;
    const int w1 = w0 + per < nwds ? w0 + per : nwds;
    int local = 0;
    for (int w = w0; w < w1; ++w) {
      if (mk.on() && words[WS * w]) words[WS * w] &= mk.word(w0lo + w);  // the output mask's exclusions
      local += __popc(words[WS * w]);
    }
    int64_t total;
    const int64_t excl = block_excl_scan(local, scratch, &total);
    if (COUNT) {
      for (int w = w0; w < w1; ++w) words[WS * w] = 0;
      if (tid == 0) gstore(P.ov_cnt + v, total);
      __syncthreads();
      return total;
    }
    if (!SR::kVal) {
      int64_t r = out_pos + excl;
      for (int w = w0; w < w1; ++w) {
        uint32_t b = words[w];
        while (b) {
          const int bit = __ffs(b) - 1;
          b &= b - 1;
          gstore(O.idx + r, lo32 + (w << 5) + bit);
          ++r;
        }
        words[w] = 0;
      }
      __syncthreads();
      return total;
    }
    {
      int run = (int)excl;
      for (int w = w0; w < w1; ++w) {
        words[WS * w + 1] = (uint32_t)run;
        run += __popc(words[WS * w]);
      }
    }
    cnt = total;
    __syncthreads();
  }
  if (mk.on()) {
    RankAcc<SR, true> accum{words, vals, lo32};
    if (RECS && rb >= 0) for_products_recs<SR>(P, rb, nrec, wid, nw, accum);
    else for_products<SR>(P, v, b0, b1, wid, nw, accum);
  } else {
    RankAcc<SR, false> accum{words, vals, lo32};
    if (RECS && rb >= 0) for_products_recs<SR>(P, rb, nrec, wid, nw, accum);
    else for_products<SR>(P, v, b0, b1, wid, nw, accum);
  }
  __syncthreads();
  // emit in three coalesced passes: the values are already dense by rank;
  // the ids are scattered by rank into the (emptied) value slots, then
  // written in rank order. Every slot is back to zero at the end.
  const int n = (int)cnt;
  for (int r = tid; r < n; r += nt) {
    gstore((T *)O.val + out_pos + r, SR::dec(vals[r]));
    vals[r] = Slot();
  }
  __syncthreads();
  int32_t *ids = (int32_t *)vals;
  if constexpr (two) {
    for (int tw = tw0; tw < tw1; ++tw) {
      uint32_t tb = top[tw];
      while (tb) {
        const int w = (tw << 5) + __ffs(tb) - 1;
        tb &= tb - 1;
        uint32_t b = words[WS * w];
        int r = (int)words[WS * w + 1];
        while (b) {
          const int bit = __ffs(b) - 1;
          b &= b - 1;
          ids[r++] = lo32 + (w << 5) + bit;
        }
        words[WS * w] = 0;
        words[WS * w + 1] = 0;
      }
      top[tw] = 0;
    }
  } else {
    for (int w = tid; w < nwds; w += nt) {
      uint32_t b = words[WS * w];
      if (b) {
        int r = (int)words[WS * w + 1];
        while (b) {
          const int bit = __ffs(b) - 1;
          b &= b - 1;
          ids[r++] = lo32 + (w << 5) + bit;
        }
      }
      words[WS * w] = 0;
      words[WS * w + 1] = 0;
    }
  }
  __syncthreads();
  for (int r = tid; r < n; r += nt) {
    gstore(O.idx + out_pos + r, ids[r]);
    ids[r] = 0;
  }
  __syncthreads();
  return cnt;
}

// Mid tier, open-addressing hash in LDS (ids stored as id + 1, 0 = empty),
// then a bitonic sort of the whole table by id.
__device__ __forceinline__ uint32_t hash_id(uint32_t id, int logts) { return (id * 0x9E3779B1u) >> (32 - logts); }

template <int K, bool COUNT>
__device__ __forceinline__ void mid_hash_vector(const Plan &P, int64_t v, uint32_t *lds, int64_t *scratch) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  typedef typename SR::Slot Slot;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wid = tid / kWave, nw = nt / kWave;
  const int64_t f = P.ov_flops[v];
  const int64_t minor = uload(&P.groups[uload(P.ov_group + v)].minor);
  const int64_t ub = f < minor ? f : minor;
  int logts = 6;
  while ((1ll << logts) < 2 * ub) ++logts;
  const int ts = 1 << logts;
  const int mask = ts - 1;
  uint32_t *keys = lds;
  Slot *vals = (Slot *)(lds + ts);

  auto ins = step<T>([&](int id, T x) {
    const uint32_t kk = (uint32_t)id + 1u;
    int h = (int)hash_id((uint32_t)id, logts);
    while (true) {
      uint32_t cur = keys[h];
      if (cur == 0) cur = atomicCAS(&keys[h], 0u, kk);
      if (cur == 0 || cur == kk) break;
      h = (h + 1) & mask;
    }
    if (!COUNT) SR::acc(&vals[h], x);
  });
  for_products<SR>(P, v, -1, -1, wid, nw, ins);
  __syncthreads();
  const MaskRef mk = mask_of(P, v);
  if (COUNT) {
    int64_t local = 0;
    for (int i = tid; i < ts; i += nt) {
      local += keys[i] != 0 && mk.keeps(keys[i] - 1u);
      keys[i] = 0;
    }
    const int64_t total = block_sum(local, scratch);
    if (tid == 0) P.ov_cnt[v] = total;
    __syncthreads();
    return;
  }
  // empty slots, and ids the output mask excludes, sort last
  for (int i = tid; i < ts; i += nt)
    if (keys[i] == 0 || !mk.keeps(keys[i] - 1u)) keys[i] = 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= ts; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (ts >> 1); i += nt) {
        const int lo = ((i / j) * 2 * j) + (i % j);
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint32_t a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
          if (SR::kVal) {
            const Slot t = vals[lo];
            vals[lo] = vals[hi];
            vals[hi] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  const OutDev O = uload(P.outs + uload(P.ov_group + v));
  const int64_t base = out_offset(P, v);
  const int64_t cnt = P.ov_cnt[v];
  for (int i = tid; i < ts; i += nt) {
    if (i < cnt) {
      gstore(O.idx + base + i, (int32_t)(keys[i] - 1u));
      if (SR::kVal) gstore((T *)O.val + base + i, SR::dec(vals[i]));
    }
    keys[i] = 0;
    vals[i] = Slot();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Heavy tier, dense LDS accumulator (flag bit + value per id) over the ids
// [lo, hi) of split bucket c. COUNT returns the number of entries.
template <int K, bool COUNT>
__device__ __forceinline__ int64_t dense_window(const Plan &P, int64_t v, int c, int64_t lo, int64_t hi, int64_t out_pos,
                                uint32_t *lds, int64_t *scratch, int wcap) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  typedef typename SR::Slot Slot;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wid = tid / kWave, nw = nt / kWave;
  const int nwf = (int)((hi - lo + 31) >> 5);
  uint32_t *flags = lds;
  Slot *vals = (Slot *)(lds + align2(wcap));
  const int lo32 = (int)lo;

  auto acc = step<T>([&](int id, T x) {
    const int r = id - lo32;
    atomicOr(&flags[r >> 5], 1u << (r & 31));
    if (!COUNT) SR::acc(&vals[r], x);
  });
  for_products<SR>(P, v, c, c + 1, wid, nw, acc);
  __syncthreads();

  const int per = (nwf + nt - 1) / nt;
  const int w0 = tid * per < nwf ? tid * per : nwf;
  const int w1 = w0 + per < nwf ? w0 + per : nwf;
  const MaskRef mk = mask_of(P, v);
  const int64_t wlo = lo >> 5;
  int local = 0;
  for (int w = w0; w < w1; ++w) {
    const uint32_t f = flags[w];
    local += __popc(mk.on() && f ? f & mk.word(wlo + w) : f);
  }
  int64_t total;
  const int64_t excl = block_excl_scan(local, scratch, &total);
  if (COUNT) {
    for (int w = w0; w < w1; ++w) flags[w] = 0;
    __syncthreads();
    return total;
  }
  const OutDev O = uload(P.outs + uload(P.ov_group + v));
  int64_t r = out_pos + excl;
  for (int w = w0; w < w1; ++w) {
    uint32_t b = flags[w];
    const uint32_t keep = mk.on() && b ? mk.word(wlo + w) : ~0u;
    while (b) {
      const int bit = __ffs(b) - 1;
      b &= b - 1;
      const int x = (w << 5) + bit;
      const bool out = (keep >> bit) & 1u;  // masked ids are only cleared
      if (out) gstore(O.idx + r, lo32 + x);
      if (SR::kVal) {
        if (out) gstore((T *)O.val + r, SR::dec(vals[x]));
        vals[x] = Slot();
      }
      r += out;
    }
    flags[w] = 0;
  }
  __syncthreads();
  return total;
}

// Count pass of one heavy vector: entries per split bucket (P.bcnt) and in
// total (ov_cnt). Mode 1 marks the whole id range once in an LDS bitmap;
// mode 0 counts bucket by bucket with the dense window.
template <int K, int MODE>
__device__ void heavy_count(const Plan &P, int64_t q, uint32_t *lds, int64_t *scratch) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t v = uload(P.heavy_list + q);
  const GroupDev G = uload(P.groups + uload(P.ov_group + v));
  int32_t *bc = P.bcnt + q * (int64_t)P.nbmax;
  if (G.mode != MODE) return;
  if (MODE == 0) {
    int64_t total = 0;
    for (int c = 0; c < G.nsplit; ++c) {
      const int64_t lo = (int64_t)c * G.sw;
      const int64_t hi = lo + G.sw < G.minor ? lo + G.sw : G.minor;
      const int64_t n = dense_window<K, true>(P, v, c, lo, hi, 0, lds, scratch, (G.sw + 31) >> 5);
      if (tid == 0) bc[c] = (int32_t)n;
      total += n;
    }
    if (tid == 0) P.ov_cnt[v] = total;
    // every item ends on a barrier after its thread-0 stores: without it the
    // compiler may let the other lanes re-enter the queue loop on their own
    __syncthreads();
    return;
  }
  const int wid = tid / kWave, nw = nt / kWave;
  const int nwds = (int)((G.minor + 31) >> 5);
  uint32_t *bits = lds;
  int32_t *lbc = (int32_t *)(lds + nwds);
  auto mark = flat_step<T>([&](int id, T) { atomicOr(&bits[id >> 5], 1u << (id & 31)); });
  for_products<SR>(P, v, -1, -1, wid, nw, mark);
  __syncthreads();
  const int wpb = G.sw >> 5;  // words per bucket
  uint32_t *keep = q < P.nkeep ? P.hbits + q * P.hstride : nullptr;
  int64_t local = 0;
  // thread t owns the contiguous words [t * per, (t + 1) * per), per a
  // multiple of 4: they are read and kept 16 bytes at a time, and their
  // popcount goes to the bucket counter with one LDS atomic per bucket run
  int per = (nwds + nt - 1) / nt;
  per = (per + 3) & ~3;
  const int w0 = tid * per < nwds ? tid * per : nwds;
  const int w1 = w0 + per < nwds ? w0 + per : nwds;
  const bool vec = ((((uintptr_t)bits) | (keep ? (uintptr_t)keep : 0)) & 15) == 0;
  const MaskRef mk = mask_of(P, v);
  int bk_run = -1, acc = 0;
  for (int w = w0; w < w1; w += 4) {
    uint32_t x[4];
    if (vec && w + 3 < w1) {
      const u32x4 q = *(const u32x4 *)&bits[w];
      x[0] = q.x;
      x[1] = q.y;
      x[2] = q.z;
      x[3] = q.w;
      if (q.x | q.y | q.z | q.w) *(u32x4 *)&bits[w] = u32x4{0u, 0u, 0u, 0u};
      if (mk.on()) {  // the output mask's exclusions leave the counts and the kept bitmap
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (x[j]) x[j] &= mk.word(w + j);
      }
      if (keep) gstore((u32x4 *)(keep + w), u32x4{x[0], x[1], x[2], x[3]});
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        x[j] = w + j < w1 ? bits[w + j] : 0u;
        if (w + j < w1) {
          if (x[j]) bits[w + j] = 0;
          if (mk.on() && x[j]) x[j] &= mk.word(w + j);
          if (keep) gstore(keep + w + j, x[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (w + j >= w1) break;
      const int c = __popc(x[j]);
      const int bk = (w + j) / wpb;
      if (bk != bk_run) {
        if (acc) atomicAdd(&lbc[bk_run], acc);
        bk_run = bk;
        acc = 0;
      }
      acc += c;
      local += c;
    }
  }
  if (acc) atomicAdd(&lbc[bk_run], acc);
  const int64_t total = block_sum(local, scratch);
  for (int b = tid; b < G.nsplit; b += nt) {
    bc[b] = lbc[b];
    lbc[b] = 0;
  }
  if (tid == 0) P.ov_cnt[v] = total;
  __syncthreads();
}

// Numeric pass of one planned heavy window (MODE 2: either window kind).
// `it` is wave-uniform; the item's descriptor is one scalar load.
template <int K, int MODE, bool RECS>
__device__ __forceinline__ void heavy_item(const Plan &P, int64_t it, uint32_t *lds, int64_t *scratch) {
  const ItemDev I = uload(P.items + it);
  const GroupDev G = uload(P.groups + I.g);
  const int64_t lo = (int64_t)I.b0 * G.sw;
  const int64_t hi = (int64_t)I.b1 * G.sw < G.minor ? (int64_t)I.b1 * G.sw : G.minor;
  if (MODE != 2 && G.mode != MODE) return;
  int64_t n;
  if (MODE == 0 || (MODE == 2 && G.mode == 0))
    n = dense_window<K, false>(P, I.v, I.b0, lo, hi, I.pos, lds, scratch, (G.sw + 31) >> 5);
  else
    n = rank_window<K, false, false, RECS>(P, I.v, lo, hi, I.b0, I.b1, I.pos, lds, scratch,
                                           I.q < P.nkeep ? P.hbits + I.q * P.hstride : nullptr, I.rbase, I.nrec);
  if constexpr (SG_CHECK) {
    if (threadIdx.x == 0) {
      const int32_t *bc = P.bcnt + (int64_t)I.q * P.nbmax;
      int64_t want = 0;
      for (int b = I.b0; b < I.b1; ++b) want += gload(bc + b);
      chk_count(P, n != want);
    }
  }
}

// Numeric pass of mid-tier vector m (position in the mid list; either
// accumulator). RECS: the plan may hold the vector's entry records, which
// both passes of the rank accumulator then walk instead of the descriptors.
template <int K, bool RECS>
__device__ __forceinline__ void mid_item(const Plan &P, int64_t m, uint32_t *lds, int64_t *scratch) {
  const int64_t v = uload(P.mid_list + m);
  if (P.mid_kind == 0) {
    const int64_t rb = RECS && P.mid_rb ? uload(P.mid_rb + m) : -1;
    const int32_t nrec = rb >= 0 ? uload(P.mid_nrec + m) : 0;
    const int64_t n = rank_window<K, false, true, RECS>(P, v, 0, uload(&P.groups[uload(P.ov_group + v)].minor), -1,
                                                        -1, out_offset(P, v), lds, scratch, nullptr, rb, nrec);
    chk_count(P, threadIdx.x == 0 && n != gload(P.ov_cnt + v));
  } else {
    mid_hash_vector<K, false>(P, v, lds, scratch);
  }
}

// ---------------------------------------------------------------------------
// Small list: a mid-tier vector of at most kSmallMaxFlops products on one
// wavefront, with no workgroup barrier. Product s of the vector (its slot)
// goes to lane s mod 64, register s / 64: its id into a register, its
// value (the S value times the G value) into the wavefront's own LDS array
// at index s. Every gather load of a half of the registers is in flight
// before the first is used. The registers then hold packed keys
// (id << 10 | slot), which a bitonic network sorts into lane-major order
// (element e = ep lane + j for the ep registers in use, ep = 1, 2, 4, 8 or
// 16, the fewest that hold the vector): a key names its value's slot, so
// only the 32-bit keys move through the network. Equal ids end up adjacent
// in slot order; their values are read back from LDS and summed in that
// order (a lane's trailing run and the segmented prefix of those across
// lanes give each lane the part of its first run held by earlier lanes),
// and each lane writes its run ends at their ranks. Padding slots hold the
// key 0xFFFFFFFF and sort last; ids stay below 2^22 - 1 (kSmallMaxMinor)
// so that no packed key reaches it. The network is a loop over its stages,
// one code block per exchange distance, not unrolled: a fully unrolled
// network is thousands of instructions, which every wavefront would stream
// through the instruction cache for each vector.
constexpr uint32_t kSmallPad = 0xFFFFFFFFu;
constexpr int kSmallSlotBits = 10;  // slots < kSmallMaxFlops

// One stage across lanes: element e and e xor (LM * EP) compare-exchange,
// ascending where e & k is 0 (the pair's lower element keeps the minimum).
// EP, the registers in use, is a template argument so that every register
// index is a constant: with a run-time count the compiler indexes the key
// array through the register file and branches per compare.
template <int EP, int LM>
__device__ __forceinline__ void small_xstage(uint32_t (&key)[kSmallPerLane], int k) {
  const int l = lane();
  const bool low = (l & LM) == 0;
#pragma unroll
  for (int j = 0; j < EP; ++j) {
    const uint32_t pk = xor_lane(key[j], LM);
    const bool up = ((l * EP + j) & k) == 0;
    const uint32_t mn = pk < key[j] ? pk : key[j], mx = pk < key[j] ? key[j] : pk;
    key[j] = low == up ? mn : mx;
  }
}
// One stage inside a lane: registers j and j + M.
template <int EP, int M>
__device__ __forceinline__ void small_istage(uint32_t (&key)[kSmallPerLane], int k) {
  const int l = lane();
#pragma unroll
  for (int j = 0; j < EP; ++j) {
    if (j & M) continue;
    const int jp = j | M;
    const bool up = ((l * EP + j) & k) == 0;
    const uint32_t a = key[j], b = key[jp];
    const uint32_t mn = a < b ? a : b, mx = a < b ? b : a;
    key[j] = up ? mn : mx;
    key[jp] = up ? mx : mn;
  }
}

// Sort and emit of a small-list vector whose products fill EP registers per
// lane: a bitonic sort of the EP x 64 packed keys into element order
// e = EP lane + j, then run ends, their ranks and (numeric) the run sums.
template <int K, bool COUNT, int EP>
__device__ __forceinline__ void small_finish(const Plan &P, int64_t v, uint32_t (&key)[kSmallPerLane],
                                             typename Sr<K>::T *wvals) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  const int l = lane();
#pragma unroll 1
  for (int k = 2; k <= EP * kWave; k <<= 1) {
#pragma unroll 1
    for (int m = k >> 1; m >= EP; m >>= 1) {
      switch (uni(m / EP)) {  // the lane distance, uniform: one code block per distance
        case 1: small_xstage<EP, 1>(key, k); break;
        case 2: small_xstage<EP, 2>(key, k); break;
        case 4: small_xstage<EP, 4>(key, k); break;
        case 8: small_xstage<EP, 8>(key, k); break;
        case 16: small_xstage<EP, 16>(key, k); break;
        default: small_xstage<EP, 32>(key, k); break;
      }
    }
    if constexpr (EP > 8) if (k >= 16) small_istage<EP, 8>(key, k);
    if constexpr (EP > 4) if (k >= 8) small_istage<EP, 4>(key, k);
    if constexpr (EP > 2) if (k >= 4) small_istage<EP, 2>(key, k);
    if constexpr (EP > 1) small_istage<EP, 1>(key, k);
  }
  // run ends: the next element (the next lane's first for the last register)
  // has another id
  const uint32_t first = key[0] >> kSmallSlotBits;
  const uint32_t idlast = key[EP - 1] >> kSmallSlotBits;
  const uint32_t nfirst = (uint32_t)__shfl_down((int)first, 1, kWave);
  const MaskRef mk = mask_of(P, v);
  uint32_t tails = 0;
#pragma unroll
  for (int j = 0; j < EP; ++j) {
    const uint32_t id = key[j] >> kSmallSlotBits;
    const uint32_t next = j + 1 < EP ? key[j + 1 < EP ? j + 1 : j] >> kSmallSlotBits
                                     : (l + 1 < kWave ? nfirst : (kSmallPad >> kSmallSlotBits));
    bool t = key[j] != kSmallPad && (next != id || (j + 1 == EP && l + 1 == kWave));
    if (mk.on() && t) t = mk.keeps((int64_t)id);
    tails |= (uint32_t)t << j;
  }
  const int cnt = __popc(tails);
  const int incl = wave_incl_scan(cnt);
  const int total = read_lane(incl, kWave - 1);
  if (COUNT) {
    if (l == 0) P.ov_cnt[v] = total;
    return;
  }
  chk_count(P, l == 0 && (int64_t)total != gload(P.ov_cnt + v));
  const OutDev O = uload(P.outs + uload(P.ov_group + v));
  int64_t pos = out_offset(P, v) + (incl - cnt);
  if (!SR::kVal) {
#pragma unroll
    for (int j = 0; j < EP; ++j)
      if ((tails >> j) & 1u) gstore(O.idx + pos++, (int32_t)(key[j] >> kSmallSlotBits));
    return;
  }
  __builtin_amdgcn_wave_barrier();  // the values were written by other lanes of this wavefront
  // the lane's trailing run (slot order), then the same across lanes
  T tail_sum = T();
  bool have = false;
#pragma unroll
  for (int j = 0; j < EP; ++j) {
    if (key[j] != kSmallPad && (key[j] >> kSmallSlotBits) == idlast) {
      const T x = wvals[key[j] & (kSmallMaxFlops - 1)];
      tail_sum = have ? SR::add(tail_sum, x) : x;
      have = true;
    }
  }
  const T run_lanes = seg_prefix<SR>((uint64_t)idlast, tail_sum);
  const uint32_t pid = (uint32_t)__shfl_up((int)idlast, 1, kWave);
  const T carry = __shfl_up(run_lanes, 1, kWave);
  const bool carried = l > 0 && pid == first && key[0] != kSmallPad;
  T run = T();
#pragma unroll
  for (int j = 0; j < EP; ++j) {
    if (key[j] == kSmallPad) break;
    const uint32_t id = key[j] >> kSmallSlotBits;
    const T x = wvals[key[j] & (kSmallMaxFlops - 1)];
    if (j == 0) run = carried ? SR::add(carry, x) : x;
    else run = id == (key[j > 0 ? j - 1 : 0] >> kSmallSlotBits) ? SR::add(run, x) : x;
    if ((tails >> j) & 1u) {
      gstore(O.idx + pos, (int32_t)id);
      gstore((T *)O.val + pos, run);
      ++pos;
    }
  }
}

// wvals: this wavefront's LDS array of kSmallMaxFlops values (unused when
// counting or without values).
template <int K, bool COUNT, bool RECS>
__device__ __forceinline__ void small_vector(const Plan &P, int64_t v, int64_t p, typename Sr<K>::T *wvals) {
  typedef Sr<K> SR;
  typedef typename SR::T T;
  constexpr int E = kSmallPerLane;
  constexpr int H = E / 2;  // registers per gather half
  constexpr bool kVals = SR::kVal && !COUNT;
  static_assert(E == 16 && kSmallMaxFlops == (1 << kSmallSlotBits), "stage blocks and slot bits below");
  const int l = lane();
  uint32_t key[E];  // gathered ids, then packed keys
#pragma unroll
  for (int j = 0; j < E; ++j) key[j] = kSmallPad;
  int filled = 0;
  // one batch of up to 64 entries, one per lane: `len` products whose ids
  // start at address ia and values at va (S value sv); products f of the
  // batch go to slots filled + f
  auto place = [&](int len, int64_t ia, int64_t va, T sv) {
    const int incl = wave_incl_scan(len);
    const int tot = read_lane(incl, kWave - 1);
    if (tot == 0) return;
    const int st = incl - len;  // the entry's first product in the batch
    const int64_t ia0 = ia - (int64_t)st * (int64_t)sizeof(int32_t);  // id address of product 0 of the entry
    const int64_t va0 = va - (int64_t)st * (int64_t)sizeof(T);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      T gv[H];
      uint32_t own[2] = {0u, 0u};  // owner lane of each register's product, 8 bits each
      uint32_t got = 0;
#pragma unroll
      for (int jj = 0; jj < H; ++jj) {
        const int j = h * H + jj;
        gv[jj] = T();
        const int f0 = j * kWave - filled;  // the batch product in this register of lane 0
        if (f0 >= tot || f0 + kWave <= 0) continue;  // uniform: no lane has a product in this register
        const int f = f0 + l;
        const bool mine = f >= 0 && f < tot;
        // the entry of each lane's product: the entry of the register's
        // first product, unless entries start later in the register (a few
        // are taken in order; many, by a binary search)
        const int r0 = f0 > 0 ? f0 : 0;
        int o = (int)__popcll(__ballot(incl <= r0));
        const uint64_t starts = __ballot(len > 0 && st > r0 && st < f0 + kWave);
        if (starts) {
          if (__popcll(starts) <= 4) {
            uint64_t m = starts;
            while (m) {
              const int x = __ffsll((unsigned long long)m) - 1;
              m &= m - 1;
              if (f >= read_lane(st, x)) o = x;
            }
          } else {
            o = owner_of(incl, mine ? f : 0);
          }
        }
        const int64_t a = __shfl(ia0, o, kWave) + (int64_t)f * (int64_t)sizeof(int32_t);
        const int64_t b = kVals ? __shfl(va0, o, kWave) + (int64_t)f * (int64_t)sizeof(T) : 0;
        own[jj >> 2] |= (uint32_t)o << (8 * (jj & 3));
        if (mine) {
          key[j] = (uint32_t)gload((const int32_t *)a);
          if (kVals) gv[jj] = gload((const T *)b);
          got |= 1u << jj;
        }
      }
      if (kVals) {
#pragma unroll
        for (int jj = 0; jj < H; ++jj) {
          const int j = h * H + jj;
          const int f0 = j * kWave - filled;
          if (f0 + kWave <= 0 || f0 >= tot) continue;  // uniform: no lane gathered into register j
          const T sj = __shfl(sv, (int)((own[jj >> 2] >> (8 * (jj & 3))) & 63u), kWave);
          if ((got >> jj) & 1u) wvals[j * kWave + l] = SR::mul(sj, gv[jj]);
        }
      }
    }
    filled += tot;
  };
  const int64_t rb = RECS && P.mid_rb ? uload(P.mid_rb + p) : -1;
  if (RECS && rb >= 0) {
    const int32_t nrec = uload(P.mid_nrec + p);
    for (int64_t eb = 0; eb < nrec; eb += kWave) {
      const int64_t x = rb + eb + l;
      const bool ok = eb + l < nrec;
      const int len = ok ? gload(P.rec_len + x) : 0;
      const int64_t gi = ok ? gload(P.rec_gi + x) : 0;
      const int64_t gv = (SR::kVal && ok) ? gload(P.rec_gv + x) : 0;
      const T sv = (SR::kVal && ok) ? gload((const T *)P.rec_sv + x) : T();
      place(len, gi, gv, sv);
    }
  } else {
    const int64_t s0 = uload(P.ov_seg + v), s1 = uload(P.ov_seg + v + 1);
    for (int64_t s = s0; s < s1; ++s) {
      const ProdDev d = uload(P.prods + uload(P.seg_prod + s));
      const int32_t t = uload(P.seg_svec + s);
      const int64_t e1 = uload(d.s_ptr + t + 1);
      for (int64_t eb = uload(d.s_ptr + t); eb < e1; eb += kWave) {
        int len;
        int64_t gb;
        T sv;
        load_entry<SR>(d, eb + l, e1, -1, -1, len, gb, sv);
        place(len, (int64_t)(d.g_idx + gb), SR::kVal ? (int64_t)((const T *)d.g_val + gb) : 0, sv);
      }
    }
  }
  // packed keys
#pragma unroll
  for (int j = 0; j < E; ++j)
    if (key[j] != kSmallPad) key[j] = (key[j] << kSmallSlotBits) | (uint32_t)(j * kWave + l);
  // registers in use: the vector's products fill ceil(filled / 64) of them,
  // rounded up to a power of two
  const int ep = filled <= kWave ? 1 : (filled <= 2 * kWave ? 2 : (filled <= 4 * kWave ? 4 : (filled <= 8 * kWave ? 8 : 16)));
  switch (uni(ep)) {
    case 1: small_finish<K, COUNT, 1>(P, v, key, wvals); break;
    case 2: small_finish<K, COUNT, 2>(P, v, key, wvals); break;
    case 4: small_finish<K, COUNT, 4>(P, v, key, wvals); break;
    case 8: small_finish<K, COUNT, 8>(P, v, key, wvals); break;
    default: small_finish<K, COUNT, 16>(P, v, key, wvals); break;
  }
}

// ---------------------------------------------------------------------------
// Kernels. Mid and heavy kernels pull work from a device queue counter;
// every workgroup exits once the counter passes the item count, which is
// fixed before the launch, so every wave reaches the exit.
__device__ __forceinline__ void zero_lds(uint32_t *lds, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) lds[i] = 0;
  __syncthreads();
}

template <int K, bool COUNT>
__global__ void __launch_bounds__(1024) k_tiny(Plan P) {
  const int64_t n = P.counters[kCtTiny];
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  // chunks as large as needed to give every wavefront work, at most 64
  const int64_t csz = tiny_chunk(n, nwaves);
  for (int64_t c0 = wave * csz; c0 < n; c0 += nwaves * csz) tiny_pack<K, COUNT>(P, c0, c0 + csz < n ? c0 + csz : n);
}

// Small-list vectors, one per wavefront at a time (count pass: COUNT; the
// numeric pass walks entry records where the plan has them).
template <int K, bool COUNT, bool RECS>
__global__ void __launch_bounds__(1024) k_small(Plan P) {
  typedef typename Sr<K>::T T;
  extern __shared__ uint32_t lds[];  // kSmallMaxFlops values per wavefront (numeric pass)
  T *wvals = (T *)lds + (threadIdx.x / kWave) * kSmallMaxFlops;
  const int64_t nm = P.counters[kCtMid];
  const int64_t n = P.counters[kCtSmall];
  const int64_t wave = uni((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wave; i < n; i += nwaves) small_vector<K, COUNT, RECS>(P, uload(P.small_list + i), nm + i, wvals);
}

template <int K>
__global__ void __launch_bounds__(kBlockMax, kWavesPerSimd) k_mid(Plan P, int64_t *queue) {
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
    mid_item<K, false>(P, i, lds, scratch);
    chk_lds_zero(P, lds);
  }
}

// MODE selects the heavy window kind this launch handles (items of groups
// with the other kind are skipped); a plan launches one kernel per kind used.
// The numeric launch keeps one queue per XCD over the windows of that XCD's id ranges
// (`queue` has kXcds counters); a workgroup starts with the queue of the XCD
// it runs on, taken as blockIdx.x mod kXcds (workgroups are dispatched to
// the dies round-robin), and then drains the others in turn. RECS: the
// plan has entry records (a separate instantiation, so plans without them
// keep the plain walk's code).
template <int K, int MODE, bool RECS>
__global__ void __launch_bounds__(kBlockMax, kWavesPerSimd) k_heavy(Plan P, int64_t *queue) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t scratch[kMaxWaves + 1];
  __shared__ int64_t s_item;
  zero_lds(lds, P.lds_words);
  const int per_xcd = P.nrange >= kXcds ? P.nrange / kXcds : 0;
  const int home = blockIdx.x % kXcds;
  for (int d = 0; d < kXcds; ++d) {
    const int x = (home + d) % kXcds;
    int64_t lo, hi;
    if (per_xcd == 0) {  // ranges off: one queue, held by XCD 0's counter
      lo = 0;
      hi = x == 0 ? P.counters[kCtItems] : 0;
    } else {
      lo = P.ibase[(int64_t)x * per_xcd * P.ibase_stride];
      hi = P.ibase[(int64_t)(x + 1) * per_xcd * P.ibase_stride];
    }
    if (lo >= hi) continue;
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long *)&queue[x], 1ull);
    __syncthreads();
    int64_t i = lo + uni(s_item);
    __syncthreads();
    while (i < hi) {
      // the next item is claimed before this one starts, so the queue's
      // round trip overlaps the window instead of preceding it
      int64_t nxt = 0;
      if (threadIdx.x == 0) nxt = (int64_t)atomicAdd((unsigned long long *)&queue[x], 1ull);
      heavy_item<K, MODE, RECS>(P, i, lds, scratch);
      chk_lds_zero(P, lds);
      if (threadIdx.x == 0) s_item = nxt;
      __syncthreads();
      i = lo + uni(s_item);
      __syncthreads();
    }
  }
}

// Count passes of the mid and heavy tiers. They need only the id bitmaps
// (no values), so they run with a smaller LDS allocation; the mid count
// pass also gets a register budget for twice the resident wavefronts of
// the numeric kernels (it is bound by the latency of its gathers).
constexpr int kCountWavesPerSimd = 8;

template <int K>
__global__ void __launch_bounds__(kBlockMax, kCountWavesPerSimd) k_mid_count(Plan P, int64_t *queue) {
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
    const int64_t v = uload(P.mid_list + i);
    if (P.mid_kind == 0) rank_window<K, true, true>(P, v, 0, uload(&P.groups[uload(P.ov_group + v)].minor), -1, -1, 0, lds, scratch);
    else mid_hash_vector<K, true>(P, v, lds, scratch);
    chk_lds_zero(P, lds);
  }
}

// The heavy count pass of rank windows (MODE 1) has the same register
// budget: its flat walk of bitmap marks fits it without spills. Dense
// windows (MODE 0) keep the numeric kernels' budget.
template <int MODE>
constexpr int heavy_count_waves() { return MODE == 1 ? kCountWavesPerSimd : kWavesPerSimd; }

template <int K, int MODE>
__global__ void __launch_bounds__(kBlockMax, heavy_count_waves<MODE>()) k_heavy_count(Plan P, int64_t *queue) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t scratch[kMaxWaves + 1];
  __shared__ int64_t s_item;
  zero_lds(lds, P.lds_words);
  const int64_t n = P.counters[kCtHeavy];
  while (true) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long *)queue, 1ull);
    __syncthreads();
    const int64_t i = uni(s_item);
    __syncthreads();
    if (i >= n) break;
    heavy_count<K, MODE>(P, i, lds, scratch);
    chk_lds_zero(P, lds);
  }
}

// One persistent launch for the workgroup tiers: queue items are heavy
// windows first, then mid vectors, then chunks of 64 tiny-list positions
// (one chunk per wavefront, packed as in tiny_pack). The small list runs in
// its own launch (k_small): its registers would otherwise count against
// every path of this kernel.
template <int K, int MODE, bool RECS>
__global__ void __launch_bounds__(kBlockMax, kWavesPerSimd) k_batched(Plan P, int64_t *queue, int64_t n_items, int64_t n_mid,
                                                  int64_t n_tiny) {
  extern __shared__ uint32_t lds[];
  __shared__ int64_t scratch[kMaxWaves + 1];
  __shared__ int64_t s_item;
  zero_lds(lds, P.lds_words);
  const int nw = blockDim.x / kWave;
  const int64_t csz = tiny_chunk(n_tiny, (int64_t)gridDim.x * nw);
  const int64_t n_tiny_groups = (n_tiny + csz * nw - 1) / (csz * nw);
  const int64_t total = n_items + n_mid + n_tiny_groups;
  while (true) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long *)queue, 1ull);
    __syncthreads();
    const int64_t i = uni(s_item);
    __syncthreads();
    if (i >= total) break;
    if (i < n_items) {
      heavy_item<K, MODE, RECS>(P, i, lds, scratch);
    } else if (i < n_items + n_mid) {
      mid_item<K, RECS>(P, i - n_items, lds, scratch);
    } else {
      const int64_t c0 = uni(((i - n_items - n_mid) * nw + threadIdx.x / kWave) * csz);
      if (c0 < n_tiny) tiny_pack<K, false>(P, c0, c0 + csz < n_tiny ? c0 + csz : n_tiny);
    }
    chk_lds_zero(P, lds);
  }
}

}  // namespace sg
