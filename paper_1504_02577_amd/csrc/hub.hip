// Panther query, hub queries of the batched form (Alg. 1 counting and the
// top-k of Problem 1 for queries with long path lists), split across many
// work-groups with every count kept on chip.
//
// A query q whose list P_q is too long for one work-group's LDS table goes
// through four steps, each a grid-wide launch over all hub queries of a
// chunk:
//   gather   rows of P_q -> their distinct vertices != q, T slots per row
//            (-1 where a row has fewer), in a staging array; each tile
//            also counts its vertices per bucket (nb buckets for query q,
//            nb = ceil(staged slots / kBucketTarget); bucket of v =
//            floor(h(v) * nb / 2^32) for a bijective 32-bit hash h, so the
//            buckets split the hash range into nb near-equal intervals),
//            keeps the tile's counts and adds them to the bucket totals;
//   bucket   the totals are scanned, and each tile moves its vertices into
//            bucket order (its run of a bucket placed by one atomic
//            reservation); a query with a single bucket skips this step,
//            its count reads the row-order staging;
//   count    one work-group per bucket counts its vertices in an LDS hash
//            table and selects the bucket's k best (count desc, id asc);
//   merge    one work-group per query selects the k best of the per-bucket
//            winners.
// Buckets partition the candidates of q, so the k best overall are among
// the per-bucket k best, and the result is exactly that of one dense count
// of q.  A bucket whose distinct vertices overflow the LDS table is redone
// in sub-ranges of its hash interval (the top bits of h(v) * nb mod 2^32,
// which runs through the interval in steps of nb), doubling the split until
// it fits; a sub-range holding at most half the table's size of hash
// values holds at most that many distinct vertices, so the doubling ends.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/panther.h"
#include "common.h"
#include "runtime.h"
#include "kernels.h"
#include "hub.h"

using namespace panther;

namespace {

constexpr int kGatherBlock = 256;
constexpr int kGatherRows = 4;                        // rows per thread
constexpr int kTileRows = kGatherBlock * kGatherRows;  // rows per gather tile
// Rows per bucketing tile: one gather tile, whose per-bucket counts the
// gather keeps for the scatter.  (Before the gather counted, 4,096-row
// bucketing tiles measured 1.5 ms slower per R-MAT 24 call than 1,024.)
constexpr int kSTileRows = kTileRows;
constexpr int kCountBlock = 1024;
constexpr int kTable = 8192;  // LDS hash entries of the count step
constexpr int kTableBits = 13;
constexpr int kProbes = 32;                // bounded probe sequence
constexpr int kFitBits = kTableBits - 1;   // log2(kTable / 2)
constexpr uint32_t kRareGrid = 256;        // work-groups of the rare count path
static_assert(kTable == 1 << kTableBits, "table size");
static_assert(kBucketTarget * 8 <= kTable * 5, "table load");

__device__ __forceinline__ uint32_t vhash(int32_t v) { return (uint32_t)v * 0x9E3779B1u; }

__device__ __forceinline__ uint32_t bucket_of(int32_t v, uint32_t nb) {
  return (uint32_t)(((uint64_t)vhash(v) * nb) >> 32);
}

// Sub-range `sub` of 2^sbits of v's bucket: the top sbits of the position
// of h(v) inside the bucket's hash interval.
__device__ __forceinline__ uint32_t sub_of(int32_t v, uint32_t nb, int sbits) {
  return (uint32_t)((uint64_t)vhash(v) * nb) >> (32 - sbits);
}

// True when a sub-range of 2^sbits holds at most kTable / 2 hash values
// (ceil(2^(32 - sbits) / nb)), hence at most that many distinct vertices.
__device__ __forceinline__ bool finest_split(uint32_t nb, int sbits) {
  return ((((uint64_t)1 << (32 - sbits)) + nb - 1) / nb) <= (uint64_t)kTable / 2;
}

// kUnroll staged slots per thread, loaded before any is used (-1 past m):
// the loads of a batch overlap instead of each waiting on the one before.
constexpr int kUnroll = 8;
__device__ __forceinline__ void load_batch(const int32_t* __restrict__ src, uint64_t m, uint64_t i0,
                                           int32_t (&x)[kUnroll]) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const uint64_t i = i0 + (uint64_t)u * kGatherBlock + threadIdx.x;
    x[u] = i < m ? src[i] : -1;
  }
}

// Per query of the chunk: its list bounds, the owner maps of its tiles and
// buckets, and zeroed bucket counters.
__global__ void __launch_bounds__(256) k_hub_prep(HubArgs A) {
  const int j = blockIdx.x;
  const HubQuery Q = A.hq[j];
  const bool last = j + 1 == A.nq;
  const uint32_t t1 = last ? A.n_tiles : A.hq[j + 1].tile0;
  const uint32_t s1 = last ? A.n_stiles : A.hq[j + 1].stile0;
  const uint32_t nb = Q.nb;
  if (threadIdx.x == 0) {
    const int32_t q = A.queries[Q.qi];
    const uint64_t a = A.inv_ptr[q];
    A.hx[j] = HubList{a, A.inv_ptr[q + 1] - a, q, 0};
    A.cand_n[j] = 0u;
  }
  for (uint32_t t = Q.tile0 + threadIdx.x; t < t1; t += 256) A.tile_owner[t] = j;
  for (uint32_t t = Q.stile0 + threadIdx.x; t < s1; t += 256) A.stile_owner[t] = j;
  for (uint32_t b = threadIdx.x; b < nb; b += 256) {
    A.bkt_owner[Q.bkt0 + b] = j;
    A.bkt_cand0[Q.bkt0 + b] = Q.cand0;
    A.bkt_cnt[Q.bkt0 + b] = 0u;
    A.bkt_fill[Q.bkt0 + b] = 0u;
  }
  if (j == 0 && threadIdx.x == 0) *A.redo_n = 0u;
}

template <int S>
__global__ void __launch_bounds__(kGatherBlock) k_hub_gather(HubArgs A) {
  __shared__ uint32_t hist[1 << kMaxBucketBits];
  const uint32_t tile = blockIdx.x;
  const int j = A.tile_owner[tile];
  const HubQuery Q = A.hq[j];
  const HubList X = A.hx[j];
  const int32_t q = X.q;
  const uint64_t a = X.a;
  const uint64_t L = X.L;
  const int T = A.T;
  const int nb = (int)Q.nb;
  const uint64_t r0 = (uint64_t)(tile - Q.tile0) * kTileRows;
  for (int b = threadIdx.x; b < nb; b += kGatherBlock) hist[b] = 0u;
  __syncthreads();
  // rows are held in registers RG at a time (fewer for long rows)
  constexpr int RG = S <= 16 ? kGatherRows : 1;
#pragma unroll 1
  for (int g0 = 0; g0 < kGatherRows; g0 += RG) {
    uint32_t pid[RG];
    bool ok[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      const uint64_t r = r0 + (uint64_t)(g0 + i) * kGatherBlock + threadIdx.x;
      ok[i] = r < L;
      pid[i] = ok[i] ? A.inv_pid[a + r] : 0u;
    }
    int32_t v[RG][S];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      if (ok[i]) {
        load_row<S>(A.paths, (uint64_t)pid[i], v[i]);
      } else {
#pragma unroll
        for (int jj = 0; jj < S; ++jj) v[i][jj] = -1;
      }
    }
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      if (!ok[i]) continue;
      dedup_row<S>(v[i]);
      const uint64_t r = r0 + (uint64_t)(g0 + i) * kGatherBlock + threadIdx.x;
      int32_t* dst = A.stA + Q.occ0 + r * (uint64_t)T;
      int c = 0;
#pragma unroll
      for (int jj = 0; jj < S; ++jj) {
        const int32_t x = v[i][jj];
        if (x >= 0 && x != q && c < T) {
          dst[c++] = x;
          atomicAdd(&hist[bucket_of(x, Q.nb)], 1u);
        }
      }
      for (int jj = c; jj < T; ++jj) dst[jj] = -1;
    }
  }
  // the tile's bucket counts: kept for the scatter, added to the totals
  __syncthreads();
  uint32_t* th = A.th + Q.th0 + (uint64_t)(tile - Q.tile0) * (uint32_t)nb;
  for (int b = threadIdx.x; b < nb; b += kGatherBlock) {
    const uint32_t h = hist[b];
    th[b] = h;
    // a single-bucket query is counted from its row-order staging: its
    // bucket keeps an empty range of the bucket order
    if (h && nb > 1) atomicAdd(&A.bkt_cnt[Q.bkt0 + b], h);
  }
}

__global__ void __launch_bounds__(kGatherBlock) k_hub_scatter(HubArgs A) {
  __shared__ uint32_t hist[1 << kMaxBucketBits];
  __shared__ uint32_t base[1 << kMaxBucketBits];
  const uint32_t tile = blockIdx.x;
  const int j = A.stile_owner[tile];
  const HubQuery Q = A.hq[j];
  if (Q.nb == 1u) return;  // its bucket is its row-order staging
  const uint64_t L = A.hx[j].L;
  const int nb = (int)Q.nb;
  const uint64_t r0 = (uint64_t)(tile - Q.stile0) * kSTileRows;
  const uint64_t rows = L - r0 < (uint64_t)kSTileRows ? L - r0 : (uint64_t)kSTileRows;
  const uint64_t m = rows * (uint64_t)A.T;
  const int32_t* src = A.stA + Q.occ0 + r0 * (uint64_t)A.T;
  // this tile's bucket counts, from the gather
  const uint32_t* th = A.th + Q.th0 + (uint64_t)(tile - Q.stile0) * (uint32_t)nb;
  for (int b = threadIdx.x; b < nb; b += kGatherBlock) {
    const uint32_t h = th[b];
    base[b] = h ? (uint32_t)A.bkt_start[Q.bkt0 + b] + atomicAdd(&A.bkt_fill[Q.bkt0 + b], h) : 0u;
    hist[b] = 0u;
  }
  __syncthreads();
  for (uint64_t i0 = 0; i0 < m; i0 += kUnroll * kGatherBlock) {
    int32_t x[kUnroll];
    load_batch(src, m, i0, x);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (x[u] >= 0) {
        const uint32_t b = bucket_of(x[u], Q.nb);
        A.stB[base[b] + atomicAdd(&hist[b], 1u)] = x[u];
      }
  }
}

// Table slot: top bits of a second multiplicative hash, so that the ids of
// one bucket (one interval of vhash) still spread over the whole table.
__device__ __forceinline__ uint32_t slot_of(int32_t v) {
  return ((uint32_t)v * 0xCC9E2D51u) >> (32 - kTableBits);
}

// Counts v in the LDS table; false when `probes` slots found no room.
__device__ __forceinline__ bool table_add(int32_t* keys, uint32_t* vals, int32_t v, int probes) {
  uint32_t h = slot_of(v);
#pragma unroll 1
  for (int p = 0; p < probes; ++p) {
    // one LDS round trip per probe: the swap claims an empty slot, and a
    // failed swap returns the slot's key
    const int32_t prev = atomicCAS(&keys[h], -1, v);
    if (prev == -1 || prev == v) {
      atomicAdd(&vals[h], 1u);
      return true;
    }
    h = (h + 1) & (uint32_t)(kTable - 1);
  }
  return false;
}

// LDS of the count step's common path: the table and a count histogram.
struct alignas(16) TableSmem {
  int32_t keys[kTable];
  uint32_t vals[kTable];
  uint32_t ch[256];
  uint32_t ctl[8];
};

// LDS of the rare path (buckets the common path hands over): the table,
// the exact block selection and the running best of the sub-ranges.
struct alignas(16) CountSmem {
  int32_t keys[kTable];
  uint32_t vals[kTable];  // the two arrays are reused as kTable 64-bit keys
  SelectSmem sel;
  uint64_t run[kOutCap];
  uint32_t ctl[8];
};

// The slots of bucket g of query j: its run [s, e) of the bucket order, or,
// for a query with a single bucket, the query's whole row-order staging
// (the scatter leaves such queries alone; -1 marks the empty slots of rows
// with fewer vertices, which the count skips).
__device__ __forceinline__ const int32_t* bucket_slots(const HubArgs& A, uint32_t g, int j,
                                                      uint64_t* s, uint64_t* e) {
  *s = A.bkt_start[g];
  *e = A.bkt_start[g + 1];
  if (*s != *e) return A.stB;
  const HubQuery Q = A.hq[j];
  if (Q.nb != 1u) return A.stB;  // an empty bucket
  *s = Q.occ0;
  *e = Q.occ0 + A.hx[j].L * (uint64_t)A.T;
  return A.stA;
}

// Counts the vertices of src[s, e) (one bucket of a query with nb buckets)
// whose sub-range of 2^sbits is `sub` (all of them when sbits == 0) in the
// LDS table.  Returns false when the table overflowed.  At the finest split
// at most kTable / 2 distinct ids qualify and the probe sequence is
// unbounded, so it never fails there.
__device__ bool count_part(const HubArgs& A, const int32_t* src, int32_t* keys, uint32_t* vals,
                           uint32_t* ctl, uint64_t s, uint64_t e, uint32_t nb, int sbits,
                           uint32_t sub) {
  const int probes = sbits > 0 && finest_split(nb, sbits) ? kTable : kProbes;
  for (int j = threadIdx.x; j < kTable / 4; j += kCountBlock) {
    reinterpret_cast<int4*>(keys)[j] = make_int4(-1, -1, -1, -1);
    reinterpret_cast<uint4*>(vals)[j] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (threadIdx.x == 0) {
    ctl[0] = 0u;
    ctl[1] = 0u;
  }
  __syncthreads();
  bool fail = false;
  for (uint64_t i0 = s; i0 < e; i0 += kUnroll * kCountBlock) {
    int32_t x[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t i = i0 + (uint64_t)u * kCountBlock + threadIdx.x;
      x[u] = i < e ? src[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (x[u] < 0) continue;
      if (sbits > 0 && sub_of(x[u], nb, sbits) != sub) continue;
      if (!table_add(keys, vals, x[u], probes)) fail = true;
    }
  }
  if (fail) ctl[1] = 1u;
  __syncthreads();
  const bool overflow = ctl[1] != 0u;
  __syncthreads();
  return !overflow;
}

// Exact selection of the k best entries of the table into sel.out (sorted);
// returns how many.
__device__ int select_exact(const HubArgs& A, CountSmem& sm) {
  // compact the occupied slots into ranking keys over the table's storage
  constexpr int kPer = kTable / kCountBlock;
  int32_t kk[kPer];
  uint32_t vv[kPer];
  int nv = 0;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    kk[t] = sm.keys[threadIdx.x + t * kCountBlock];
    vv[t] = sm.vals[threadIdx.x + t * kCountBlock];
    nv += kk[t] >= 0 ? 1 : 0;
  }
  if (threadIdx.x == 0) sm.ctl[0] = 0u;
  __syncthreads();
  const uint32_t p0 = nv ? atomicAdd(&sm.ctl[0], (uint32_t)nv) : 0u;
  __syncthreads();
  uint64_t* comp = reinterpret_cast<uint64_t*>(sm.keys);
  uint32_t p = p0;
#pragma unroll
  for (int t = 0; t < kPer; ++t)
    if (kk[t] >= 0) comp[p++] = rank_key(vv[t], kk[t]);
  __syncthreads();
  const int nc = (int)sm.ctl[0];
  auto keyfn = [&](int i) { return comp[i]; };
  return block_select_topk<kCountBlock>(keyfn, nc, A.k, sm.sel);
}

// Emits, unsorted, every entry of the table whose count reaches the count
// of the k-th best entry (all entries when there are fewer than k): a
// superset of the bucket's k best, since the ranking puts larger counts
// first.  Returns false, emitting nothing, when that set exceeds
// max(k, kEmitCap) entries.
__device__ bool emit_by_count(const HubArgs& A, TableSmem& sm, int j, uint64_t cand0) {
  constexpr int kBins = 256;  // counts clamped to 255
  constexpr int kPer = kTable / kCountBlock;  // table slots per thread
  static_assert(kPer == 8, "two 16-byte loads per array");
  for (int b = threadIdx.x; b < kBins; b += kCountBlock) sm.ch[b] = 0u;
  if (threadIdx.x == 0) {
    sm.ctl[2] = 1u;  // threshold count (when there are fewer than k entries)
    sm.ctl[3] = 0u;  // entries at or above it
    sm.ctl[4] = 0u;  // emit cursor
  }
  // each thread keeps its eight consecutive slots in registers for both
  // passes over the table
  int32_t kk[kPer];
  uint32_t cc[kPer];
  {
    const int4* k4 = reinterpret_cast<const int4*>(sm.keys) + 2 * threadIdx.x;
    const uint4* c4 = reinterpret_cast<const uint4*>(sm.vals) + 2 * threadIdx.x;
    const int4 a0 = k4[0], a1 = k4[1];
    const uint4 b0 = c4[0], b1 = c4[1];
    kk[0] = a0.x; kk[1] = a0.y; kk[2] = a0.z; kk[3] = a0.w;
    kk[4] = a1.x; kk[5] = a1.y; kk[6] = a1.z; kk[7] = a1.w;
    cc[0] = b0.x; cc[1] = b0.y; cc[2] = b0.z; cc[3] = b0.w;
    cc[4] = b1.x; cc[5] = b1.y; cc[6] = b1.z; cc[7] = b1.w;
  }
  __syncthreads();
  // counts 1..3 (most entries) are summed per wave in three 10-bit fields
  // (at most kPer per lane, 512 per wave) and added once per wave; larger
  // counts go straight to their bin
  static_assert(kPer * kWave < 1024, "10-bit fields");
  uint32_t low = 0u;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    if (kk[i] >= 0) {
      const uint32_t c = cc[i];
      if (c - 1u < 3u)
        low += 1u << (10u * (c - 1u));
      else
        atomicAdd(&sm.ch[c < kBins - 1 ? c : kBins - 1], 1u);
    }
  }
  low = __ockl_wfred_add_u32(low);  // wave sum (DPP lane moves)
  if ((threadIdx.x & (kWave - 1)) == 0 && low) {
    atomicAdd(&sm.ch[1], low & 1023u);
    atomicAdd(&sm.ch[2], (low >> 10) & 1023u);
    atomicAdd(&sm.ch[3], low >> 20);
  }
  __syncthreads();
  // the threshold, by one wave: lane L holds bins 255 - 4L .. 252 - 4L
  // (descending), a wave scan gives the entries above each of them
  const uint32_t k = (uint32_t)A.k;
  const int lane = threadIdx.x & (kWave - 1);
  static_assert(kBins == 4 * kWave, "four bins per lane");
  if (threadIdx.x < kWave) {
    uint32_t hb[4], sum = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      hb[i] = sm.ch[kBins - 1 - 4 * lane - i];
      sum += hb[i];
    }
    const uint32_t inc = wave_inclusive_sum(sum);
    uint32_t above = inc - sum;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int bin = kBins - 1 - 4 * lane - i;
      if (bin >= 1 && above < k && above + hb[i] >= k) {
        sm.ctl[2] = (uint32_t)bin;
        sm.ctl[3] = above + hb[i];
      }
      above += hb[i];
    }
    if (lane == kWave - 1) sm.ctl[6] = inc;  // entries in the table
  }
  __syncthreads();
  const uint32_t thr = sm.ctl[2];
  const uint32_t tot = sm.ctl[6];
  const uint32_t n_emit = tot < k ? tot : sm.ctl[3];
  const uint32_t cap = (uint32_t)(A.k > kEmitCap ? A.k : kEmitCap);
  if (n_emit > cap) return false;  // uniform: every thread read the same words
  if (threadIdx.x == 0) sm.ctl[5] = n_emit ? atomicAdd(&A.cand_n[j], n_emit) : 0u;
  // a wave's emitted entries: ballots first, then one cursor add per wave
  uint64_t mask[kPer];
  uint32_t wtot = 0u;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    mask[i] = __ballot(kk[i] >= 0 && (cc[i] < kBins - 1 ? cc[i] : kBins - 1) >= thr);
    wtot += (uint32_t)__popcll(mask[i]);
  }
  uint32_t base = 0u;
  if (lane == 0 && wtot) base = atomicAdd(&sm.ctl[4], wtot);
  base = __builtin_amdgcn_readfirstlane(base);  // lane 0's value (all lanes active)
  __syncthreads();
  uint64_t* dst = A.cand + cand0 + sm.ctl[5];
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    if ((mask[i] >> lane) & 1ull) dst[base + __popcll(mask[i] & below)] = rank_key(cc[i], kk[i]);
    base += (uint32_t)__popcll(mask[i]);
  }
  return true;
}

// Common path: one work-group of 1,024 threads per bucket; its table
// (64 KB) lets two work-groups share a CU at eight waves per SIMD.  A
// work-group's life is mostly a few dependent memory round trips (bucket
// bounds, its slots, the winners' cursor), so buckets are made as large as
// that occupancy allows: halving them measured slower.  A bucket whose
// table overflows, or whose candidate superset exceeds the emit cap, is
// handed to k_hub_count_rare.
__global__ void __launch_bounds__(kCountBlock) k_hub_count(HubArgs A) {
  __shared__ TableSmem sm;
  const uint32_t g = blockIdx.x;
  const int j = A.bkt_owner[g];
  const uint64_t cand0 = A.bkt_cand0[g];
  uint64_t s, e;
  const int32_t* src = bucket_slots(A, g, j, &s, &e);
  if (count_part(A, src, sm.keys, sm.vals, sm.ctl, s, e, 1u, 0, 0u) &&
      emit_by_count(A, sm, j, cand0))
    return;
  if (threadIdx.x == 0) A.redo[atomicAdd(A.redo_n, 1u)] = g;
}

// Rare path, a fixed grid looping over the handed-over buckets: exact
// selection, and recounting in hash sub-ranges when the table overflowed.
__global__ void __launch_bounds__(kCountBlock) k_hub_count_rare(HubArgs A) {
  extern __shared__ __align__(16) char lds[];
  CountSmem& sm = *reinterpret_cast<CountSmem*>(lds);
  const uint32_t nredo = *A.redo_n;
  for (uint32_t r = blockIdx.x; r < nredo; r += gridDim.x) {
    const uint32_t g = A.redo[r];
    const int j = A.bkt_owner[g];
    const HubQuery Q = A.hq[j];
    uint64_t s, e;
    const int32_t* src = bucket_slots(A, g, j, &s, &e);
    int m;
    const uint64_t* best = sm.sel.out;
    if (count_part(A, src, sm.keys, sm.vals, sm.ctl, s, e, Q.nb, 0, 0u)) {
      m = select_exact(A, sm);
    } else {
      // split by the next hash bits until every part fits
      m = 0;
      for (int sbits = 1; sbits <= 32 - kFitBits; ++sbits) {
        int rr = 0;  // keys in sm.run
        bool ok = true;
        for (uint32_t sub = 0; sub < (1u << sbits); ++sub) {
          if (!count_part(A, src, sm.keys, sm.vals, sm.ctl, s, e, Q.nb, sbits, sub)) {
            ok = false;
            break;
          }
          const int mm = select_exact(A, sm);
          // merge sel.out[0..mm) into run[0..rr): both descending, keep k
          uint64_t* buf = sm.sel.cand;
          const int tot = rr + mm;
          const int P = next_pow2(tot < 2 ? 2 : tot);
          for (int i = threadIdx.x; i < P; i += kCountBlock)
            buf[i] = i < rr ? sm.run[i] : (i < tot ? sm.sel.out[i - rr] : 0ull);
          __syncthreads();
          block_bitonic_desc<kCountBlock>(buf, P);
          rr = tot < A.k ? tot : A.k;
          for (int i = threadIdx.x; i < rr; i += kCountBlock) sm.run[i] = buf[i];
          __syncthreads();
        }
        if (ok) {
          m = rr;
          best = sm.run;
          break;
        }
      }
    }
    // the finest split holds at most kTable / 2 distinct ids, so m is set
    if (threadIdx.x == 0) sm.ctl[5] = m > 0 ? atomicAdd(&A.cand_n[j], (uint32_t)m) : 0u;
    __syncthreads();
    const uint32_t pos = sm.ctl[5];
    for (int i = threadIdx.x; i < m; i += kCountBlock) A.cand[Q.cand0 + pos + i] = best[i];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kCountBlock) k_hub_merge(HubArgs A) {
  extern __shared__ __align__(16) char lds[];
  SelectSmem& sm = *reinterpret_cast<SelectSmem*>(lds);
  const int j = blockIdx.x;
  const HubQuery Q = A.hq[j];
  const int n = (int)A.cand_n[j];
  const uint64_t* c = A.cand + Q.cand0;
  auto keyfn = [&](int i) { return c[i]; };
  const int m = block_select_topk<kCountBlock>(keyfn, n, A.k, sm);
  const int k = A.k;
  const int64_t row = (int64_t)Q.qi * k;
  if (A.theta) {
    for (int i = threadIdx.x; i < k; i += kCountBlock)
      A.theta[row + i] = i < m ? (float)key_count(sm.out[i]) / A.fR : 0.0f;
    return;
  }
  for (int i = threadIdx.x; i < k; i += kCountBlock) {
    const bool ok = i < m;
    A.out_ids[row + i] = ok ? key_vertex(sm.out[i]) : -1;
    A.out_counts[row + i] = ok ? key_count(sm.out[i]) : 0u;
  }
  if (threadIdx.x == 0) A.out_len[Q.qi] = m;
}

}  // namespace

namespace panther {

uint32_t hub_buckets(uint64_t occ, int max_bits) {
  const uint64_t lim = (uint64_t)1 << std::min(std::max(max_bits, 0), kMaxBucketBits);
  const uint64_t nb = (occ + kBucketTarget - 1) / kBucketTarget;
  return (uint32_t)std::max<uint64_t>(1, std::min(nb, lim));
}

uint32_t hub_tiles(uint64_t L) { return (uint32_t)((L + kTileRows - 1) / kTileRows); }
uint32_t hub_stiles(uint64_t L) { return (uint32_t)((L + kSTileRows - 1) / kSTileRows); }

size_t hub_count_lds() { return sizeof(CountSmem); }

// Enqueues the four steps for one chunk.  Buffers in `A` must hold the
// chunk's totals; nothing here allocates or synchronises.
hipError_t enqueue_hub_chunk(const HubArgs& A, int stride, void* scan_temp, hipStream_t s) {
  if (A.nq == 0) return hipSuccess;
  k_hub_prep<<<(uint32_t)A.nq, 256, 0, s>>>(A);
  switch (stride) {
    case 4: k_hub_gather<4><<<A.n_tiles, kGatherBlock, 0, s>>>(A); break;
    case 8: k_hub_gather<8><<<A.n_tiles, kGatherBlock, 0, s>>>(A); break;
    case 16: k_hub_gather<16><<<A.n_tiles, kGatherBlock, 0, s>>>(A); break;
    case 32: k_hub_gather<32><<<A.n_tiles, kGatherBlock, 0, s>>>(A); break;
    default: k_hub_gather<64><<<A.n_tiles, kGatherBlock, 0, s>>>(A); break;
  }
  launch_scan_u32_to_u64(A.bkt_cnt, A.bkt_start, A.n_bkt, scan_temp, s);
  k_hub_scatter<<<A.n_stiles, kGatherBlock, 0, s>>>(A);
  k_hub_count<<<A.n_bkt, kCountBlock, 0, s>>>(A);
  k_hub_count_rare<<<A.n_bkt < kRareGrid ? A.n_bkt : kRareGrid, kCountBlock, sizeof(CountSmem),
                     s>>>(A);
  k_hub_merge<<<(uint32_t)A.nq, kCountBlock, sizeof(SelectSmem), s>>>(A);
  return hipGetLastError();
}

hipError_t hub_set_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_hub_count_rare,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(CountSmem));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_hub_merge, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)sizeof(SelectSmem));
}

}  // namespace panther
