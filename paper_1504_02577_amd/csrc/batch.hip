// Panther query, batched form: every query of a call in one launch
// sequence (captured in a HIP graph and replayed), with the tile sizes
// picked by an autotuner.
//
// Queries are split by the length L of their path list P_q (known on the
// host from the index offsets) into three tiers, each ordered longest
// length class first:
//   A  (T*L fits half of a per-wave LDS table): one wavefront per query in
//      k_topk_waves.  Open-addressing hash (vertex -> count) in LDS, then
//      the occupied slots are compacted to 64-bit ranking keys and
//      bitonic-sorted by the wave alone (no work-group barrier).
//   B  (fits half of a work-group LDS table): one work-group per query in
//      the persistent k_topk_batched (work queue), LDS hash, then block
//      selection of the k largest keys.
//   C  (hubs, the rest): split across many work-groups by the pipeline in
//      hub.hip (candidates bucketed by a hash of their id, each bucket
//      counted in LDS by its own work-group, per-bucket winners merged),
//      on a second stream beside the other two.
// Counting is exact integer arithmetic and the ranking key (count desc, id
// asc) is a total order, so the result equals the plain form bit for bit.
#include <fcntl.h>
#include <sys/file.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/panther.h"
#include "common.h"
#include "runtime.h"
#include "hub.h"
#include "kernels.h"

using namespace panther;

namespace {

constexpr int kQueueCtl = 4;  // [0] work-queue head

// A tier item as the kernels read it: the list P_q = inv_pid[a, a + L) of
// query q (batch index qi), expanded once per call after planning, so that
// a query costs one dependent load before its list instead of three (item,
// query, offsets).
struct ItemRec {
  uint64_t a;
  uint32_t L;
  int32_t qi;
  int32_t q;
  int32_t pad;
};

struct BatchArgs {
  const int32_t* queries;  // [nq]
  const ItemRec* itemsB;   // the B queries, longest class first
  const ItemRec* itemsA;
  int32_t nB, nA;
  // tier A runs in four phases of 64, 32, 16 and 8 lanes per query:
  // itemsA [0, nA64), [nA64, nA32), [nA32, nA16), [nA16, nA)
  int32_t nA64, nA32, nA16;
  const uint64_t* inv_ptr;
  const uint32_t* inv_pid;
  const int32_t* paths;
  uint32_t* queue;         // kQueueCtl words
  int32_t n;
  int32_t k;
  int32_t TB;              // tier B table size (a power of two)
  int32_t* out_ids;
  uint32_t* out_counts;
  int32_t* out_len;
  // feature mode (Panther++): row qi of theta gets count / R of the k = D
  // largest counts, zero-padded; out_ids/out_counts/out_len unused
  float* theta;
  float fR;
};

__device__ __forceinline__ uint32_t hash_slot(int32_t v, uint32_t mask) {
  return ((uint32_t)v * 0x9E3779B1u >> 7) & mask;
}

// LDS hash insert (vertex -> +1).  The tier bounds keep the load at most
// 1/2, so a free slot always exists; the probe count is capped anyway so
// that no input can make the loop run forever.
__device__ __forceinline__ void lds_insert(int32_t* keys, uint32_t* vals, uint32_t mask,
                                           int32_t v) {
  uint32_t h = hash_slot(v, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const int32_t cur = *((volatile int32_t*)&keys[h]);
    if (cur == v) {
      atomicAdd(&vals[h], 1u);
      return;
    }
    if (cur == -1) {
      const int32_t prev = atomicCAS(&keys[h], -1, v);
      if (prev == -1 || prev == v) {
        atomicAdd(&vals[h], 1u);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Gathers the rows of P_q [a, a+L) with `nthr` threads (thread id `t`),
// calling f(v) for every distinct vertex v != q of every row.
template <int S, typename F>
__device__ __forceinline__ void for_each_candidate(const BatchArgs& A, int32_t q, uint64_t a,
                                                   uint64_t L, int t, int nthr, F&& f) {
  for (uint64_t i = t; i < L; i += nthr) {
    int32_t v[S];
    load_row<S>(A.paths, A.inv_pid[a + i], v);
    dedup_row<S>(v);
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (v[j] >= 0 && v[j] != q) f(v[j]);
  }
}

__device__ __forceinline__ void write_row(const BatchArgs& A, int32_t qi, const uint64_t* keys,
                                          int m, int t, int nthr) {
  const int k = A.k;
  if (A.theta) {
    for (int j = t; j < k; j += nthr)
      A.theta[(int64_t)qi * k + j] = j < m ? (float)key_count(keys[j]) / A.fR : 0.0f;
    return;
  }
  for (int j = t; j < k; j += nthr) {
    const bool ok = j < m;
    A.out_ids[(int64_t)qi * k + j] = ok ? key_vertex(keys[j]) : -1;
    A.out_counts[(int64_t)qi * k + j] = ok ? key_count(keys[j]) : 0u;
  }
  if (t == 0) A.out_len[qi] = m;
}

// ---- tier A: a group of G lanes of one wavefront per query (G = 64, 32,
// 16 or 8), with a table of kWaveTA * G / 64 entries ----
constexpr int kWaveTA = 512;  // table entries of a whole wave

// Item ai (< hi) of itemsA by the G lanes of this thread's group, whose LDS
// region holds 12 * TG bytes: the table (TG keys, TG counts), then up to
// TG / 2 ranking keys.  Open-addressing hash (vertex -> count), then the
// occupied slots are compacted and bitonic-sorted by the group alone (no
// work-group barrier; groups of one wave diverge only in trip counts and
// touch disjoint regions).  An inactive group (ai >= hi) writes nothing.
template <int S, int G>
__device__ void group_query(const BatchArgs& A, int ai, int hi, char* region) {
  constexpr int TG = kWaveTA * G / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const uint64_t gmask = G == kWave ? ~0ull : ((1ull << (G & 63)) - 1ull) << gbase;
  int32_t* keys = reinterpret_cast<int32_t*>(region);
  uint32_t* vals = reinterpret_cast<uint32_t*>(keys + TG);
  uint64_t* sorted = reinterpret_cast<uint64_t*>(vals + TG);  // TG/2 entries
  const bool active = ai < hi;
  int32_t qi = 0, q = -1;
  uint64_t a = 0, L = 0;
  if (active) {
    const ItemRec r = A.itemsA[ai];
    qi = r.qi;
    q = r.q;
    a = r.a;
    L = r.L;
  }
  for (int j = gl; j < TG; j += G) {
    keys[j] = -1;
    vals[j] = 0u;
  }
  wave_sync();
  for_each_candidate<S>(A, q, a, L, gl, G,
                        [&](int32_t v) { lds_insert(keys, vals, (uint32_t)TG - 1u, v); });
  wave_sync();
  // compact occupied slots into ranking keys
  int nc = 0;
  for (int base = 0; base < TG; base += G) {
    const int j = base + gl;
    const int32_t key = keys[j];
    const bool occ = key >= 0;
    const uint64_t bm = (__ballot(occ) & gmask) >> gbase;
    if (occ) sorted[nc + __popcll(bm & ((1ull << gl) - 1ull))] = rank_key(vals[j], key);
    nc += __popcll(bm);
  }
  int P = 2;
  while (P < nc) P <<= 1;
  for (int j = nc + gl; j < P; j += G) sorted[j] = 0ull;
  wave_sync();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = gl; i < (P >> 1); i += G) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi2 = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t x = sorted[lo], y = sorted[hi2];
        if ((x < y) == desc) {
          sorted[lo] = y;
          sorted[hi2] = x;
        }
      }
      wave_sync();
    }
  }
  if (active) write_row(A, qi, sorted, nc < A.k ? nc : A.k, gl, G);
  wave_sync();
}

// Items [lo, hi) in groups of G lanes: wave wg of W takes the 64 / G items
// from lo + (wg + i * W) * (64 / G) on, one per group.
template <int S, int G>
__device__ void group_items(const BatchArgs& A, int lo, int hi, int wg, int W, char* region) {
  constexpr int per = kWave / G;
  const int gi = (int)(threadIdx.x & (kWave - 1)) / G;
  char* mine = region + (size_t)gi * 12 * (kWaveTA / per);
  for (int base = lo + wg * per; base < hi; base += W * per)
    group_query<S, G>(A, base + gi, hi, mine);
}

// ---- tier B: one work-group per query, LDS table ----

// Exact top k of a tier-B query's nc ranking keys comp[0, nc) without
// sorting all of them.  A histogram of the counts gives the k-th best count
// c (keys with a larger count are certainly selected); when c is shared by
// many keys, a histogram of the top eight bits of their ids gives the digit
// holding the one whose id ranks last among the selected (ties of a smaller
// digit have smaller ids, so they are certainly selected too).  Only the
// keys at or above both thresholds survive; up to kWaveSort of them are
// sorted by one wave, with no work-group barrier.  Returns the number
// selected, sorted descending in sm.out, or -1 when more than kFastCand
// keys survive or k is large (the caller then runs the full selection);
// the answer is the same either way, since the ranking key is a total
// order.
constexpr int kFastCand = 512;
constexpr int kWaveSort = 128;
template <int BLOCK>
__device__ int select_fast(const BatchArgs& A, const uint64_t* comp, int nc, SelectSmem& sm,
                           uint32_t* s_ctl) {
  const int k = A.k;
  if (2 * k > kFastCand) return -1;  // uniform
  uint32_t* ch = sm.hist;        // 256 count bins, counts >= 255 in the last
  uint32_t* ih = sm.hist + 256;  // 256 bins of id >> s2
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t n = (uint32_t)A.n;
  const int s2 = n > 256u ? 32 - __clz((int)(n - 1u)) - 8 : 0;
  uint32_t thr = 0u, dstar = 255u;  // every key survives
  if (nc > kWaveSort) {
    for (int b = threadIdx.x; b < 512; b += BLOCK) sm.hist[b] = 0u;
    if (threadIdx.x == 0) {
      s_ctl[1] = 0u;    // threshold count
      s_ctl[2] = 0u;    // keys with a larger count
      s_ctl[4] = 255u;  // id digit threshold
      s_ctl[6] = 0u;    // ties of a smaller digit
    }
    __syncthreads();
    // counts 1 and 2 (most keys) by ballots, one add per wave
    for (int i0 = 0; i0 < nc; i0 += BLOCK) {
      const int i = i0 + (int)threadIdx.x;
      const uint32_t c = i < nc ? key_count(comp[i]) : 0u;
      const uint32_t n1 = (uint32_t)__popcll(__ballot(c == 1u));
      const uint32_t n2 = (uint32_t)__popcll(__ballot(c == 2u));
      if (lane == 0) {
        if (n1) atomicAdd(&ch[1], n1);
        if (n2) atomicAdd(&ch[2], n2);
      }
      if (c >= 3u) atomicAdd(&ch[c < 255u ? c : 255u], 1u);
    }
    __syncthreads();
    // the k-th best count (nc > k), by one wave: lane L holds bins
    // 255 - 4L .. 252 - 4L
    if (threadIdx.x < kWave) {
      uint32_t hb[4], sum = 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        hb[i] = ch[255 - 4 * lane - i];
        sum += hb[i];
      }
      uint32_t above = wave_inclusive_sum(sum) - sum;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int bin = 255 - 4 * lane - i;
        if (bin >= 1 && above < (uint32_t)k && above + hb[i] >= (uint32_t)k) {
          s_ctl[1] = (uint32_t)bin;
          s_ctl[2] = above;
        }
        above += hb[i];
      }
    }
    __syncthreads();
    thr = s_ctl[1];
    const uint32_t above = s_ctl[2];
    if (thr >= 255u) return -1;  // the k-th count is clamped: uniform
    if (above + ch[thr] > (uint32_t)kWaveSort) {
      for (int i = threadIdx.x; i < nc; i += BLOCK) {
        const uint64_t x = comp[i];
        if (key_count(x) == thr) atomicAdd(&ih[(uint32_t)key_vertex(x) >> s2], 1u);
      }
      __syncthreads();
      // the digit of the (k - above)-th smallest tie id, ascending digits
      if (threadIdx.x < kWave) {
        const uint32_t r = (uint32_t)k - above;
        uint32_t hb[4], sum = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hb[i] = ih[4 * lane + i];
          sum += hb[i];
        }
        uint32_t below = wave_inclusive_sum(sum) - sum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (below < r && below + hb[i] >= r) {
            s_ctl[4] = (uint32_t)(4 * lane + i);
            s_ctl[6] = below;
          }
          below += hb[i];
        }
      }
      __syncthreads();
      dstar = s_ctl[4];
      if (above + s_ctl[6] + ih[dstar] > (uint32_t)kFastCand) return -1;  // uniform
    }
  }
  // the survivors, by ballots with one cursor add per wave
  if (threadIdx.x == 0) s_ctl[5] = 0u;
  __syncthreads();
  uint64_t* cand = sm.cand;
  for (int i0 = 0; i0 < nc; i0 += BLOCK) {
    const int i = i0 + (int)threadIdx.x;
    const uint64_t x = i < nc ? comp[i] : 0ull;
    const uint32_t c = key_count(x);
    const bool ok =
        i < nc && (c > thr || (c == thr && ((uint32_t)key_vertex(x) >> s2) <= dstar));
    const uint64_t bm = __ballot(ok);
    uint32_t base = 0u;
    if (lane == 0 && bm) base = atomicAdd(&s_ctl[5], (uint32_t)__popcll(bm));
    base = __shfl(base, 0);
    if (ok) cand[base + __popcll(bm & ((1ull << lane) - 1ull))] = x;
  }
  __syncthreads();
  const int m = (int)s_ctl[5];
  const int P = next_pow2(m < 2 ? 2 : m);
  const int mk = m < k ? m : k;
  if (P <= kWaveSort) {
    if (threadIdx.x < kWave) {
      for (int i = m + lane; i < P; i += kWave) cand[i] = 0ull;
      wave_sync();
      for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          for (int i = lane; i < (P >> 1); i += kWave) {
            const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));
            const int hi = lo + stride;
            const bool desc = (lo & size) == 0;
            const uint64_t x = cand[lo], y = cand[hi];
            if ((x < y) == desc) {
              cand[lo] = y;
              cand[hi] = x;
            }
          }
          wave_sync();
        }
      }
      for (int i = lane; i < mk; i += kWave) sm.out[i] = cand[i];
    }
  } else {
    for (int i = m + threadIdx.x; i < P; i += BLOCK) cand[i] = 0ull;
    __syncthreads();
    block_bitonic_desc<BLOCK>(cand, P);
    for (int i = threadIdx.x; i < mk; i += BLOCK) sm.out[i] = cand[i];
  }
  __syncthreads();
  return mk;
}

template <int BLOCK, int S>
__device__ void block_query_lds(const BatchArgs& A, const ItemRec& r, char* region,
                                SelectSmem& sm, uint32_t* s_ctl) {
  const int TB = A.TB;
  int32_t* keys = reinterpret_cast<int32_t*>(region);
  uint32_t* vals = reinterpret_cast<uint32_t*>(keys + TB);
  uint64_t* comp = reinterpret_cast<uint64_t*>(vals + TB);  // TB/2 entries
  const int32_t qi = r.qi;
  const int32_t q = r.q;
  const uint64_t a = r.a;
  const uint64_t L = r.L;
  for (int j = threadIdx.x; j < TB; j += BLOCK) {
    keys[j] = -1;
    vals[j] = 0u;
  }
  if (threadIdx.x == 0) s_ctl[0] = 0u;
  __syncthreads();
  const uint32_t mask = (uint32_t)TB - 1u;
  for_each_candidate<S>(A, q, a, L, threadIdx.x, BLOCK,
                        [&](int32_t v) { lds_insert(keys, vals, mask, v); });
  __syncthreads();
  // compact: one cursor add per wave and pass (ballot ranks inside it)
  const int lane = threadIdx.x & (kWave - 1);
  for (int j = threadIdx.x; j < TB; j += BLOCK) {
    const int32_t key = keys[j];
    const uint64_t bm = __ballot(key >= 0);
    uint32_t base = 0u;
    if (lane == 0 && bm) base = atomicAdd(&s_ctl[0], (uint32_t)__popcll(bm));
    base = __shfl(base, 0);
    if (key >= 0) comp[base + __popcll(bm & ((1ull << lane) - 1ull))] = rank_key(vals[j], key);
  }
  __syncthreads();
  const int nc = (int)s_ctl[0];
  int m = select_fast<BLOCK>(A, comp, nc, sm, s_ctl);
  if (m < 0) {
    auto keyfn = [&](int i) { return comp[i]; };
    m = block_select_topk<BLOCK>(keyfn, nc, A.k, sm);
  }
  write_row(A, qi, sm.out, m, threadIdx.x, BLOCK);
  __syncthreads();
}

// ---- tier B: a persistent grid of work-groups takes the B items from a
// work queue, one query per work-group at a time ----
template <int BLOCK, int S>
__global__ void __launch_bounds__(BLOCK) k_topk_batched(BatchArgs A) {
  extern __shared__ __align__(16) char lds[];
  SelectSmem& sm = *reinterpret_cast<SelectSmem*>(lds);
  uint32_t* s_ctl = reinterpret_cast<uint32_t*>(lds + sizeof(SelectSmem));
  char* region = lds + sizeof(SelectSmem) + 64;
  while (true) {
    if (threadIdx.x == 0) {
      const uint32_t x = atomicAdd(&A.queue[0], 1u);
      s_ctl[1] = (int)x < A.nB ? x : 0xFFFFFFFFu;
    }
    __syncthreads();
    const int item = (int)s_ctl[1];
    __syncthreads();
    if (item < 0) break;
    block_query_lds<BLOCK, S>(A, A.itemsB[item], region, sm, s_ctl + 4);
  }
}

// ---- tier A as a kernel of its own: no block selection scratch, so more
// waves share a CU (six work-groups of four waves).  The A items are
// ordered longest class first; each phase (64, 32, 16, then 8 lanes per
// query) deals its items over all waves in turn, so every wave gets a
// similar mix, with no shared queue to contend on ----
constexpr int kWaveBlock = 256;
constexpr int kWaveWgsPerCu = 6;  // 6 x 24 KB of LDS per CU

template <int S>
__global__ void __launch_bounds__(kWaveBlock) k_topk_waves(BatchArgs A) {
  __shared__ __align__(16) char lds[kWaveBlock / kWave * 12 * kWaveTA];
  const int w = threadIdx.x / kWave;
  char* region = lds + (size_t)w * 12 * kWaveTA;
  const int W = (int)(gridDim.x * (kWaveBlock / kWave));
  const int wg = (int)(blockIdx.x * (kWaveBlock / kWave)) + w;
  group_items<S, 64>(A, 0, A.nA64, wg, W, region);
  group_items<S, 32>(A, A.nA64, A.nA32, wg, W, region);
  group_items<S, 16>(A, A.nA32, A.nA16, wg, W, region);
  group_items<S, 8>(A, A.nA16, A.nA, wg, W, region);
}

// ---- device planning of large batches ----
// Digit of query i in the plan's order: tier B classes 64..0 (digits
// 0..64), tier A classes 64..0 (65..129), then the hubs by class, 64..0
// (130..194); a stable sort by digit gives the host planner's tier order,
// and the hubs longest class first (the host planner orders them exactly
// by length, so that repeated queries of one vertex run side by side; the
// batches planned here, such as a pass over every vertex, rarely repeat
// one).  Also writes the pair count the sort reads and the query index as
// the sort's value.
constexpr uint32_t kHubDigit = 130;
constexpr uint32_t kDigits = kHubDigit + 65;
__global__ void k_plan_digits(const uint64_t* __restrict__ qlen, int64_t nq, uint64_t LA,
                              uint64_t LB, uint32_t* __restrict__ keys,
                              uint32_t* __restrict__ vals, uint64_t* __restrict__ nnz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *nnz = (uint64_t)nq;
  if (i >= nq) return;
  const uint64_t L = qlen[i];
  const uint32_t cl = L ? 64u - (uint32_t)__clzll((long long)L) : 0u;
  keys[i] = (L > LB ? kHubDigit : (L > LA ? 0u : 65u)) + (64u - cl);
  vals[i] = (uint32_t)i;
}

// starts[d] = first position of digit d in the sorted order, d = 0..kDigits
// (offsets are the digit-major exclusive scan of the tile counts).
__global__ void k_plan_starts(const uint64_t* __restrict__ offs, uint64_t ntiles,
                              uint64_t* __restrict__ starts) {
  const uint32_t d = threadIdx.x;
  if (d <= kDigits) starts[d] = offs[(uint64_t)d * ntiles];
}

__global__ void k_plan_hub_lengths(const int32_t* __restrict__ idx, int64_t n,
                                   const uint64_t* __restrict__ qlen, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = qlen[idx[i]];
}

__global__ void k_expand_items(const int32_t* __restrict__ items, int64_t n,
                               const int32_t* __restrict__ queries,
                               const uint64_t* __restrict__ inv_ptr, ItemRec* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t qi = items[i];
  const int32_t q = queries[qi];
  const uint64_t a = inv_ptr[q];
  out[i] = ItemRec{a, (uint32_t)(inv_ptr[q + 1] - a), qi, q, 0};
}

__global__ void k_reset_queue(uint32_t* q) {
  if (threadIdx.x < kQueueCtl) q[threadIdx.x] = 0u;
}

using KernelFn = void (*)(BatchArgs);

KernelFn pick_wave_kernel(int stride) {
  switch (stride) {
    case 4: return k_topk_waves<4>;
    case 8: return k_topk_waves<8>;
    case 16: return k_topk_waves<16>;
    case 32: return k_topk_waves<32>;
    default: return k_topk_waves<64>;
  }
}

template <int BLOCK>
KernelFn pick_kernel(int stride) {
  switch (stride) {
    case 4: return k_topk_batched<BLOCK, 4>;
    case 8: return k_topk_batched<BLOCK, 8>;
    case 16: return k_topk_batched<BLOCK, 16>;
    case 32: return k_topk_batched<BLOCK, 32>;
    default: return k_topk_batched<BLOCK, 64>;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchConfig {
  int block = 512;      // threads per work-group
  int wgs_per_cu = 1;   // persistent work-groups per CU
  int tier_b_div = 1;   // tier B keeps lists up to (LDS table bound) / tier_b_div
  int bucket_bias = 0;  // a hub query gets 2^bias times the buckets its length asks for
};

// Every value the tuner may pick; results are identical for all of them.
constexpr int kBlocks[] = {512, 256};
constexpr int kWgs[] = {1, 2};
constexpr int kTierBDivs[] = {1, 2};
constexpr int kBucketBiases[] = {0, 1};
constexpr int64_t kStage2MaxQueries = (int64_t)1 << 18;  // batches the second stage tunes

// What one call enqueues: the hub pipeline chunk by chunk, then the
// persistent kernel over tiers A and B.
struct Plan {
  BatchArgs args{};
  bool run_kernel = false;
  int stride = 0;  // path row stride: selects the kernel specialisations
  std::vector<HubArgs> hub;
  bool operator==(const Plan& o) const {
    if (run_kernel != o.run_kernel || stride != o.stride || hub.size() != o.hub.size())
      return false;
    if (std::memcmp(&args, &o.args, sizeof(args)) != 0) return false;
    for (size_t i = 0; i < hub.size(); ++i)
      if (std::memcmp(&hub[i], &o.hub[i], sizeof(HubArgs)) != 0) return false;
    return true;
  }
};

struct BatchState {
  // device plan buffers (grown as needed)
  int32_t* d_items = nullptr;
  size_t items_cap = 0;
  ItemRec* d_irec = nullptr;  // the tier items expanded (k_expand_items)
  size_t irec_cap = 0;
  uint32_t* d_queue = nullptr;
  // hub pipeline buffers (grown as needed)
  HubQuery* d_hq = nullptr;
  size_t hq_cap = 0;
  int32_t* d_stA = nullptr;
  size_t occ_cap = 0;
  int32_t* d_stB = nullptr;
  size_t occB_cap = 0;
  uint32_t* d_bkt_cnt = nullptr;
  size_t bkt_cap = 0;
  uint32_t* d_bkt_fill = nullptr;
  size_t bkt_fill_cap = 0;
  uint64_t* d_bkt_start = nullptr;
  size_t bkt_start_cap = 0;
  uint64_t* d_cand = nullptr;
  size_t cand_cap = 0;
  HubList* d_hx = nullptr;
  size_t hx_cap = 0;
  int32_t* d_tile_owner = nullptr;
  size_t tile_owner_cap = 0;
  uint32_t* d_th = nullptr;
  size_t th_cap = 0;
  int32_t* d_stile_owner = nullptr;
  size_t stile_owner_cap = 0;
  int32_t* d_bkt_owner = nullptr;
  size_t bkt_owner_cap = 0;
  uint64_t* d_bkt_cand0 = nullptr;
  size_t bkt_cand0_cap = 0;
  uint32_t* d_redo = nullptr;
  size_t redo_cap = 0;
  uint32_t* d_cand_n = nullptr;
  size_t cand_n_cap = 0;
  char* d_scan = nullptr;
  size_t scan_cap = 0;
  // page-locked staging of the plan; `uploaded` guards its reuse
  PinnedBuf pin_items, pin_hq;
  // device planning of large batches: digit keys, the sort's scratch, the
  // digit starts and the hubs' lengths (and their pinned copies)
  uint32_t* dp_keys = nullptr;
  uint32_t* dp_keys2 = nullptr;
  uint32_t* dp_vals = nullptr;
  size_t dp_cap = 0, dp_keys2_cap = 0, dp_vals_cap = 0;
  uint32_t* dp_hist = nullptr;
  size_t dp_hist_cap = 0;
  uint64_t* dp_offs = nullptr;
  size_t dp_offs_cap = 0;
  char* dp_scan = nullptr;
  size_t dp_scan_cap = 0;
  uint64_t* dp_small = nullptr;  // [0]: the pair count, [1, 133): digit starts
  size_t dp_small_cap = 0;
  uint64_t* dp_hubL = nullptr;
  size_t dp_hubL_cap = 0;
  PinnedBuf pin_starts, pin_hubL, pin_hubI;
  hipEvent_t uploaded = nullptr;
  bool upload_pending = false;
  // second stream: the hub pipeline runs beside the persistent kernel
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  size_t hub_budget = 0;  // staging budget in bytes, fixed at first use
  size_t hub_budget_forced = 0;  // option test.hub_budget (0 = automatic)
  // configuration
  bool tuned = false;
  BatchConfig cfg;
  int forced_block = 0;
  int forced_wgs = 0;
  int forced_div = 0;    // 0: chosen by the tuner
  int forced_bias = -1;  // -1: chosen by the tuner
  int64_t tier_a_override = -1;
  int64_t tier_b_override = -1;
  int hub_bits_max = 12;
  // graph cache
  hipGraphExec_t exec = nullptr;
  hipStream_t exec_stream = nullptr;
  Plan exec_plan;
  int exec_block = 0, exec_grid = 0;
  size_t exec_lds = 0;
  // the previous direct launch (a repeat of it gets captured)
  bool last_valid = false;
  hipStream_t last_stream = nullptr;
  Plan last_plan;
  int last_block = 0, last_grid = 0;
  size_t last_lds = 0;
  std::vector<std::pair<uint64_t, int32_t>> hub_sort_tmp;  // host scratch of the hub order
  std::string tune_key;
  bool no_tune = false;  // serving lanes reuse a stored or default configuration
  bool no_fork = false;  // serving lanes: one stream each (lanes overlap one another)
};

static BatchState* state(Lane* lane) {
  if (!lane->batch) lane->batch = new BatchState();
  return lane->batch;
}

void copy_batch_options(panther_ctx* c, Lane* dst) {
  BatchState* a = state(&c->lane0);
  BatchState* b = state(dst);
  b->forced_block = a->forced_block;
  b->forced_wgs = a->forced_wgs;
  b->forced_div = a->forced_div;
  b->forced_bias = a->forced_bias;
  b->tier_a_override = a->tier_a_override;
  b->tier_b_override = a->tier_b_override;
  b->hub_bits_max = a->hub_bits_max;
  b->hub_budget_forced = a->hub_budget_forced;
  b->tuned = false;
  b->no_tune = true;
  b->no_fork = true;
}

void forget_batch_graph(Lane* lane) {
  BatchState* b = lane->batch;
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->last_valid = false;
}

void free_batch_state(Lane* lane) {
  if (!lane->batch) return;
  BatchState* b = lane->batch;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->side) (void)hipStreamDestroy(b->side);
  pinned_release(b->pin_items);
  pinned_release(b->pin_hq);
  pinned_release(b->pin_starts);
  pinned_release(b->pin_hubL);
  pinned_release(b->pin_hubI);
  for (void* p : {(void*)b->dp_keys, (void*)b->dp_keys2, (void*)b->dp_vals, (void*)b->dp_hist,
                  (void*)b->dp_offs, (void*)b->dp_scan, (void*)b->dp_small, (void*)b->dp_hubL})
    ctx_free(p);
  ctx_free(b->d_items);
  ctx_free(b->d_irec);
  ctx_free(b->d_queue);
  for (void* p : {(void*)b->d_hq, (void*)b->d_stA, (void*)b->d_stB, (void*)b->d_bkt_cnt,
                  (void*)b->d_bkt_fill, (void*)b->d_bkt_start, (void*)b->d_cand,
                  (void*)b->d_cand_n, (void*)b->d_scan, (void*)b->d_hx,
                  (void*)b->d_tile_owner, (void*)b->d_stile_owner, (void*)b->d_bkt_owner,
                  (void*)b->d_bkt_cand0, (void*)b->d_redo, (void*)b->d_th})
    ctx_free(p);
  delete b;
  lane->batch = nullptr;
}

int set_batch_option(panther_ctx* c, const std::string& key, int64_t value) {
  BatchState* b = state(&c->lane0);
  if (key == "batch.block") {
    if (value != 0 && value != 256 && value != 512)
      return ctx_fail(c, PANTHER_EINVAL, "batch.block must be 0 (auto), 256 or 512");
    b->forced_block = (int)value;
  } else if (key == "batch.tier_a") {
    b->tier_a_override = value;
  } else if (key == "batch.tier_b") {
    b->tier_b_override = value;
  } else if (key == "batch.hub_bits") {
    if (value < -1 || value > 12) return ctx_fail(c, PANTHER_EINVAL, "batch.hub_bits in -1..12");
    b->hub_bits_max = value < 0 ? 12 : (int)value;
  } else if (key == "test.hub_budget") {
    if (value < 0) return ctx_fail(c, PANTHER_EINVAL, "test.hub_budget must be >= 0");
    b->hub_budget_forced = (size_t)value;
  } else if (key == "batch.wgs_per_cu") {
    if (value < 0 || value > 2) return ctx_fail(c, PANTHER_EINVAL, "batch.wgs_per_cu in 0..2");
    b->forced_wgs = (int)value;
  } else if (key == "batch.tier_b_div") {
    if (value < 0 || value > 2) return ctx_fail(c, PANTHER_EINVAL, "batch.tier_b_div in 0..2");
    b->forced_div = (int)value;
  } else if (key == "batch.bucket_bias") {
    if (value < -1 || value > 1) return ctx_fail(c, PANTHER_EINVAL, "batch.bucket_bias in -1..1");
    b->forced_bias = (int)value;
  }
  b->tuned = false;
  return PANTHER_OK;
}

namespace {

struct Layout {
  size_t lds;
  int TA, TB;
};

// LDS carve-up for a configuration: selection buffers, control words, and
// a region holding either the work-group table (12 * TB bytes: keys, counts,
// compacted keys) or one table per wave (12 * TA bytes each).
Layout layout_for(const panther_ctx* c, const BatchConfig& cfg) {
  size_t limit = (size_t)c->lds_per_block;
  if (limit > 163840) limit = 163840;
  if (cfg.wgs_per_cu > 1) limit = std::min(limit, (size_t)163840 / cfg.wgs_per_cu);
  const size_t fixed = sizeof(SelectSmem) + 64;
  const size_t avail = limit > fixed ? limit - fixed : 0;
  int TB = 64;
  while ((size_t)12 * (TB * 2) <= avail && TB < 16384) TB *= 2;
  // tier A runs in k_topk_waves with tables of its own size
  return Layout{fixed + (size_t)12 * TB, kWaveTA, TB};
}

// The configurations a lane may run: every tuner choice, with the forced
// options fixed.
std::vector<BatchConfig> config_space(const BatchState* b) {
  std::vector<BatchConfig> v;
  for (int blk : kBlocks)
    for (int wgs : kWgs)
      for (int div : kTierBDivs)
        for (int bias : kBucketBiases) {
          if ((b->forced_block && blk != b->forced_block) ||
              (b->forced_wgs && wgs != b->forced_wgs) || (b->forced_div && div != b->forced_div) ||
              (b->forced_bias >= 0 && bias != b->forced_bias))
            continue;
          v.push_back(BatchConfig{blk, wgs, div, bias});
        }
  return v;
}

std::string tune_cache_path() {
  const char* p = getenv("PANTHER_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/panther_tune.txt";
}

}  // namespace

// The cache is a text file of "key value..." lines, the values integers.
// Readers take a shared and writers an exclusive flock(2) on it, so lanes
// and processes that tune at once never interleave a line.  Every failure
// (no home, read-only disk) leaves tuning to run again next time.
std::vector<std::vector<int>> tune_cache_read(const std::string& key) {
  std::vector<std::vector<int>> out;
  const int fd = open(tune_cache_path().c_str(), O_RDONLY | O_CLOEXEC);
  if (fd < 0) return out;
  if (flock(fd, LOCK_SH) == 0) {
    std::string text;
    char buf[4096];
    ssize_t r;
    while ((r = read(fd, buf, sizeof buf)) > 0) text.append(buf, (size_t)r);
    std::istringstream lines(text);
    std::string line;
    while (std::getline(lines, line)) {
      std::istringstream is(line);
      std::string k;
      if (!(is >> k) || k != key) continue;
      std::vector<int> v;
      int x;
      while (is >> x) v.push_back(x);
      if (is.fail() && !is.eof()) continue;  // a field that is not an integer
      out.push_back(v);
    }
    (void)flock(fd, LOCK_UN);
  }
  close(fd);
  return out;
}

void tune_cache_append(const std::string& key, const std::vector<int>& fields) {
  const std::string path = tune_cache_path();
  // create the parent directories one component at a time (no shell)
  for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
    (void)mkdir(path.substr(0, pos).c_str(), 0755);
  const int fd = open(path.c_str(), O_WRONLY | O_CREAT | O_APPEND | O_CLOEXEC, 0644);
  if (fd < 0) return;
  if (flock(fd, LOCK_EX) == 0) {
    std::string line = key;
    for (int x : fields) line += " " + std::to_string(x);
    line += "\n";
    (void)!write(fd, line.data(), line.size());
    (void)flock(fd, LOCK_UN);
  }
  close(fd);
}

namespace {

// Batched-form lines: "key block wgs_per_cu tier_b_div bucket_bias" (last
// valid match wins; the last two fields may be missing, and a line with a
// value outside the tuner's choices is ignored).
bool tune_lookup(const std::string& key, BatchConfig* cfg) {
  bool found = false;
  auto one_of = [](int v, const int* xs, size_t nx) {
    return std::find(xs, xs + nx, v) != xs + nx;
  };
  for (const std::vector<int>& f : tune_cache_read(key)) {
    if (f.size() != 2 && f.size() != 4) continue;
    const int blk = f[0], wgs = f[1], div = f.size() == 4 ? f[2] : 1, bias = f.size() == 4 ? f[3] : 0;
    if (!one_of(blk, kBlocks, 2) || !one_of(wgs, kWgs, 2) || !one_of(div, kTierBDivs, 2) ||
        !one_of(bias, kBucketBiases, 2))
      continue;
    *cfg = BatchConfig{blk, wgs, div, bias};
    found = true;
  }
  return found;
}

void tune_store(const std::string& key, const BatchConfig& cfg) {
  tune_cache_append(key, {cfg.block, cfg.wgs_per_cu, cfg.tier_b_div, cfg.bucket_bias});
}

}  // namespace

// Grows a device buffer to hold at least `want` elements of `elem` bytes.
template <typename P>
static int grow(panther_ctx* c, P*& ptr, size_t& cap, size_t want, size_t elem, const char* what) {
  if (cap >= want) return PANTHER_OK;
  ctx_free(ptr);
  ptr = nullptr;
  cap = 0;
  void* p;
  const int st = ctx_alloc(c, &p, std::max<size_t>(want, 1) * elem, what);
  if (st) return st;
  ptr = static_cast<P*>(p);
  cap = std::max<size_t>(want, 1);
  return PANTHER_OK;
}

// Enqueues a plan on stream s: the hub chunks, then the persistent kernel.
// When both parts have work, the hub chunks go to a second stream forked
// from s and joined back, so they overlap the persistent kernel.
static hipError_t enqueue(panther_ctx* c, BatchState* b, const Plan& P, KernelFn fn, int grid,
                          int block, size_t lds, hipStream_t s) {
  const bool fork = !P.hub.empty() && P.run_kernel && !b->no_fork;
  hipStream_t hs = s;
  if (fork) {
    hipError_t e = hipEventRecord(b->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
    if (e != hipSuccess) return e;
    hs = b->side;
  }
  for (const HubArgs& h : P.hub) {
    const hipError_t e = enqueue_hub_chunk(h, c->stride, b->d_scan, hs);
    if (e != hipSuccess) return e;
  }
  if (P.run_kernel) {
    if (P.args.nB > 0) {
      k_reset_queue<<<1, 64, 0, s>>>(P.args.queue);
      hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, P.args);
    }
    if (P.args.nA > 0) {
      const int wgrid = c->num_cus * kWaveWgsPerCu;
      hipLaunchKernelGGL(pick_wave_kernel(c->stride), dim3(wgrid), dim3(kWaveBlock), 0, s,
                         P.args);
    }
  }
  if (fork) {
    hipError_t e = hipEventRecord(b->ev_join, b->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join, 0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// One launch of a prepared plan (a graph replay when it repeats).
static int launch_batched(panther_ctx* c, BatchState* b, const BatchConfig& cfg, const Plan& P,
                          hipStream_t s, bool use_graph) {
  const Layout lay = layout_for(c, cfg);
  const int grid = c->num_cus * cfg.wgs_per_cu;
  KernelFn fn = cfg.block == 256 ? pick_kernel<256>(c->stride) : pick_kernel<512>(c->stride);
  int st = ctx_hip(c, hipFuncSetAttribute((const void*)fn,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lay.lds),
                   "batched kernel attribute");
  if (st) return st;
  if (!P.hub.empty()) {
    st = ctx_hip(c, hub_set_attributes(), "hub kernel attributes");
    if (st) return st;
    if (!b->side && !b->no_fork) {
      st = ctx_hip(c, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "hub stream");
      if (!st) st = ctx_hip(c, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "hub events");
      if (!st) st = ctx_hip(c, hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming), "hub events");
      if (st) return st;
    }
  }
  const bool same = b->exec && b->exec_stream == s && b->exec_block == cfg.block &&
                    b->exec_grid == grid && b->exec_lds == lay.lds && b->exec_plan == P;
  if (use_graph && same) return ctx_hip(c, hipGraphLaunch(b->exec, s), "batched graph replay");
  // capture only once the same launch comes back: a graph pays off for
  // repeated identical batches, not for a stream of different ones
  const bool repeat = b->last_valid && b->last_stream == s && b->last_block == cfg.block &&
                      b->last_grid == grid && b->last_lds == lay.lds && b->last_plan == P;
  b->last_valid = true;
  b->last_stream = s;
  b->last_block = cfg.block;
  b->last_grid = grid;
  b->last_lds = lay.lds;
  b->last_plan = P;
  if (use_graph && repeat) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    hipStream_t cs;
    st = ctx_hip(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    if (st) return st;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t el = enqueue(c, b, P, fn, grid, cfg.block, lay.lds, cs);
      e = hipStreamEndCapture(cs, &graph);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    st = ctx_hip(c, e, "batched graph capture");
    if (st) return st;
    b->exec_stream = s;
    b->exec_block = cfg.block;
    b->exec_grid = grid;
    b->exec_lds = lay.lds;
    b->exec_plan = P;
    return ctx_hip(c, hipGraphLaunch(b->exec, s), "batched graph launch");
  }
  return ctx_hip(c, enqueue(c, b, P, fn, grid, cfg.block, lay.lds, s), "batched kernel");
}

// Splits the hub queries (longest first) into chunks whose staging fits a
// memory budget, and fills the device buffers and per-chunk arguments.
static int plan_hubs(panther_ctx* c, BatchState* b,
                     const std::vector<std::pair<uint64_t, int32_t>>& C,
                     const int32_t* dq, int32_t k, int bias, int32_t* d_ids, uint32_t* d_counts,
                     int32_t* d_len, float* theta, hipStream_t s, std::vector<HubArgs>* out) {
  out->clear();
  if (C.empty()) return PANTHER_OK;
  const uint64_t T = (uint64_t)c->T;
  // the plan is written straight into the pinned upload buffer (the
  // previous plan's upload has completed: plan waits for it)
  int st;
  if ((st = pinned_ensure(c, b->pin_hq, sizeof(HubQuery) * C.size(), "hub plan"))) return st;
  HubQuery* hq = static_cast<HubQuery*>(b->pin_hq.p);
  size_t nhq = 0;
  if (!b->hub_budget) {
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    b->hub_budget = std::max<size_t>(std::min((size_t)16 << 30, free_b / 4), (size_t)1 << 28);
  }
  // staging bytes per occurrence slot: row order, bucket order
  const size_t budget = b->hub_budget_forced ? b->hub_budget_forced : b->hub_budget;
  // the longest hub leads its class (exact order) or its class leads
  // (device-planned batches): it is among the first class's entries
  uint64_t max_L = 0;
  {
    const auto cls = [](uint64_t L) { return 64 - __builtin_clzll(L); };
    const int c0 = cls(C.front().first);
    for (size_t i = 0; i < C.size() && cls(C[i].first) == c0; ++i)
      max_L = std::max(max_L, C[i].first);
  }
  uint64_t occ_limit = std::max<uint64_t>(budget / 8, T * max_L);
  occ_limit = std::min<uint64_t>(occ_limit, (uint64_t)1 << 31);
  if (T * max_L > occ_limit)
    return ctx_fail(c, PANTHER_ERANGE, "a hub query's path list exceeds the staging limit");
  struct Chunk {
    size_t first, nq;
    uint32_t tiles, stiles, bkts;
    uint64_t occ, cand, ths;
  };
  std::vector<Chunk> chunks;
  Chunk cur{0, 0, 0, 0, 0, 0, 0, 0};
  size_t max_bkt = 0, max_nq = 0, max_tiles = 0, max_stiles = 0;
  uint64_t max_occ = 0, max_cand = 0, max_ths = 0;
  auto close = [&]() {
    if (!cur.nq) return;
    chunks.push_back(cur);
    max_bkt = std::max<size_t>(max_bkt, cur.bkts);
    max_nq = std::max<size_t>(max_nq, cur.nq);
    max_tiles = std::max<size_t>(max_tiles, cur.tiles);
    max_stiles = std::max<size_t>(max_stiles, cur.stiles);
    max_occ = std::max(max_occ, cur.occ);
    max_cand = std::max(max_cand, cur.cand);
    max_ths = std::max(max_ths, cur.ths);
    cur = Chunk{nhq, 0, 0, 0, 0, 0, 0, 0};
  };
  for (const auto& x : C) {
    const uint64_t L = x.first;
    const uint64_t occ = T * L;
    const uint32_t nb = hub_buckets(occ << bias, b->hub_bits_max);
    const uint32_t tiles = hub_tiles(L);
    const uint32_t stiles = hub_stiles(L);
    const uint64_t cand = std::min<uint64_t>((uint64_t)std::max(k, kEmitCap) * nb, occ);
    if (cur.nq && (cur.occ + occ > occ_limit || (uint64_t)cur.tiles + tiles > 0x7FFFFFFFu ||
                   (uint64_t)cur.nq + 1 > 0x7FFFFFFFu ||
                   (uint64_t)cur.bkts + nb > 0x7FFFFFFFu ||
                   cur.ths + (uint64_t)stiles * nb > 0xFFFFFFFFu))
      close();
    HubQuery h{};
    h.qi = x.second;
    h.nb = nb;
    h.tile0 = cur.tiles;
    h.stile0 = cur.stiles;
    h.bkt0 = cur.bkts;
    h.occ0 = cur.occ;
    h.cand0 = cur.cand;
    h.th0 = (uint32_t)cur.ths;
    hq[nhq++] = h;
    cur.nq += 1;
    cur.tiles += tiles;
    cur.stiles += stiles;
    cur.bkts += nb;
    cur.occ += occ;
    cur.cand += cand;
    cur.ths += (uint64_t)stiles * nb;
  }
  close();
  if ((st = grow(c, b->d_hq, b->hq_cap, nhq, sizeof(HubQuery), "hub plan"))) return st;
  if ((st = grow(c, b->d_stA, b->occ_cap, max_occ, sizeof(int32_t), "hub staging"))) return st;
  if ((st = grow(c, b->d_stB, b->occB_cap, max_occ, sizeof(int32_t), "hub staging"))) return st;
  if ((st = grow(c, b->d_bkt_cnt, b->bkt_cap, max_bkt, sizeof(uint32_t), "hub buckets"))) return st;
  if ((st = grow(c, b->d_bkt_fill, b->bkt_fill_cap, max_bkt, sizeof(uint32_t), "hub buckets")))
    return st;
  if ((st = grow(c, b->d_bkt_start, b->bkt_start_cap, max_bkt + 1, sizeof(uint64_t),
                 "hub buckets")))
    return st;
  if ((st = grow(c, b->d_cand, b->cand_cap, max_cand, sizeof(uint64_t), "hub winners"))) return st;
  if ((st = grow(c, b->d_cand_n, b->cand_n_cap, max_nq, sizeof(uint32_t), "hub winners")))
    return st;
  if ((st = grow(c, b->d_scan, b->scan_cap, scan_temp_bytes((int64_t)max_bkt), 1, "hub scan")))
    return st;
  if ((st = grow(c, b->d_hx, b->hx_cap, max_nq, sizeof(HubList), "hub lists"))) return st;
  if ((st = grow(c, b->d_tile_owner, b->tile_owner_cap, max_tiles, sizeof(int32_t), "hub maps")))
    return st;
  if ((st = grow(c, b->d_stile_owner, b->stile_owner_cap, max_stiles, sizeof(int32_t),
                 "hub maps")))
    return st;
  if ((st = grow(c, b->d_bkt_owner, b->bkt_owner_cap, max_bkt, sizeof(int32_t), "hub maps")))
    return st;
  if ((st = grow(c, b->d_bkt_cand0, b->bkt_cand0_cap, max_bkt, sizeof(uint64_t), "hub maps")))
    return st;
  if ((st = grow(c, b->d_redo, b->redo_cap, max_bkt + 16, sizeof(uint32_t), "hub maps")))
    return st;
  if ((st = grow(c, b->d_th, b->th_cap, max_ths, sizeof(uint32_t), "hub tile counts")))
    return st;
  st = ctx_hip(c, hipMemcpyAsync(b->d_hq, b->pin_hq.p, sizeof(HubQuery) * nhq,
                                 hipMemcpyHostToDevice, s),
               "hub plan upload");
  if (st) return st;
  for (const Chunk& ch : chunks) {
    HubArgs h{};
    h.queries = dq;
    h.inv_ptr = c->d_inv_ptr;
    h.inv_pid = c->d_inv_pid;
    h.paths = c->d_paths;
    h.hq = b->d_hq + ch.first;
    h.hx = b->d_hx;
    h.tile_owner = b->d_tile_owner;
    h.stile_owner = b->d_stile_owner;
    h.bkt_owner = b->d_bkt_owner;
    h.bkt_cand0 = b->d_bkt_cand0;
    h.redo = b->d_redo;
    h.redo_n = b->d_redo + max_bkt;
    h.nq = (int32_t)ch.nq;
    h.T = c->T;
    h.k = k;
    h.n_tiles = ch.tiles;
    h.n_stiles = ch.stiles;
    h.n_bkt = ch.bkts;
    h.stA = b->d_stA;
    h.stB = b->d_stB;
    h.bkt_cnt = b->d_bkt_cnt;
    h.bkt_start = b->d_bkt_start;
    h.bkt_fill = b->d_bkt_fill;
    h.th = b->d_th;
    h.cand = b->d_cand;
    h.cand_n = b->d_cand_n;
    h.out_ids = d_ids;
    h.out_counts = d_counts;
    h.out_len = d_len;
    h.theta = theta;
    h.fR = (float)c->R;
    out->push_back(h);
  }
  return PANTHER_OK;
}

// Orders hub queries by list length, longest first; equal lengths keep
// their order (ascending batch index).  A stable LSD radix sort on the
// length's 11-bit digits, complemented so that longer lists come first:
// linear in the number of hubs (a comparison sort of the tens of thousands
// of hubs of an R-MAT 24 batch took milliseconds of host time).
// Large sets split each pass over host threads: thread t takes a
// contiguous range, and its run of digit d starts after every earlier
// thread's run of d (positions are prefix sums in (digit, thread) order), so
// the result is the one-thread order.
static void sort_hubs_longest_first(std::vector<std::pair<uint64_t, int32_t>>& C,
                                    std::vector<std::pair<uint64_t, int32_t>>& tmp) {
  if (C.size() < 2) return;
  uint64_t max_L = 0;
  for (const auto& x : C) max_L = std::max(max_L, x.first);
  const int bits = max_L ? 64 - __builtin_clzll(max_L) : 0;
  constexpr int kDigit = 11;
  constexpr uint64_t kMask = (1u << kDigit) - 1u;
  tmp.resize(C.size());
  const size_t n = C.size();
  const int nth = n >= ((size_t)1 << 16) ? 8 : 1;
  std::vector<std::vector<size_t>> pos(nth, std::vector<size_t>(kMask + 1));
  auto lo_of = [&](int t) { return n * (size_t)t / (size_t)nth; };
  auto in_threads = [&](auto&& fn) {
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(fn, t);
    fn(0);
    for (auto& x : th) x.join();
  };
  for (int sh = 0; sh < bits; sh += kDigit) {
    in_threads([&](int t) {
      auto& pt = pos[t];
      std::fill(pt.begin(), pt.end(), (size_t)0);
      for (size_t i = lo_of(t), e = lo_of(t + 1); i < e; ++i)
        ++pt[kMask - ((C[i].first >> sh) & kMask)];
    });
    size_t run = 0;
    for (uint64_t d = 0; d <= kMask; ++d)
      for (int t = 0; t < nth; ++t) {
        const size_t c = pos[t][d];
        pos[t][d] = run;
        run += c;
      }
    in_threads([&](int t) {
      auto& pt = pos[t];
      for (size_t i = lo_of(t), e = lo_of(t + 1); i < e; ++i)
        tmp[pt[kMask - ((C[i].first >> sh) & kMask)]++] = C[i];
    });
    C.swap(tmp);
  }
}

// Device planning of a large batch: the digits of k_plan_digits sorted by
// one stable pass of the index's radix sort (8-bit digit, query index as
// the value) straight into d_items, so the tier items need no host pass and
// no upload.  Only the digit starts and the hubs' lengths come back.
// Fills nB, need (tier items), cntA (tier A items per length class) and C
// (the hubs, in batch order).
bool batched_plan_on_device(int64_t nq) { return nq >= ((int64_t)1 << 20); }

static int plan_on_device(panther_ctx* c, BatchState* b, const uint64_t* dqlen, int64_t nq,
                          uint64_t LA, uint64_t LB, hipStream_t s, bool with_hubs, size_t* nB,
                          size_t* need, std::array<size_t, 65>& cntA,
                          std::vector<std::pair<uint64_t, int32_t>>* C) {
  const uint64_t n = (uint64_t)nq;
  const uint64_t ntiles = radix_tiles_pairs(n);
  const size_t nh = (size_t)256 * ntiles;
  constexpr size_t kStarts = kDigits + 1;
  static_assert(kDigits < 256, "one 8-bit radix pass");
  int st;
  if ((st = grow(c, b->dp_keys, b->dp_cap, n, sizeof(uint32_t), "batch plan")) ||
      (st = grow(c, b->dp_keys2, b->dp_keys2_cap, n, sizeof(uint32_t), "batch plan")) ||
      (st = grow(c, b->dp_vals, b->dp_vals_cap, n, sizeof(uint32_t), "batch plan")) ||
      (st = grow(c, b->d_items, b->items_cap, std::max<size_t>(n, 1024), sizeof(int32_t),
                 "batch plan")) ||
      (st = grow(c, b->dp_hist, b->dp_hist_cap, nh, sizeof(uint32_t), "batch plan")) ||
      (st = grow(c, b->dp_offs, b->dp_offs_cap, nh + 1, sizeof(uint64_t), "batch plan")) ||
      (st = grow(c, b->dp_scan, b->dp_scan_cap, scan_temp_bytes((int64_t)nh), 1, "batch plan")) ||
      (st = grow(c, b->dp_small, b->dp_small_cap, 1 + kStarts, sizeof(uint64_t), "batch plan")) ||
      (st = pinned_ensure(c, b->pin_starts, sizeof(uint64_t) * kStarts, "batch plan")))
    return st;
  uint64_t* d_nnz = b->dp_small;
  uint64_t* d_starts = b->dp_small + 1;
  k_plan_digits<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dqlen, nq, LA, LB, b->dp_keys,
                                                            b->dp_vals, d_nnz);
  launch_radix_up_pairs(b->dp_keys, d_nnz, n, 0, 8, b->dp_hist, s);
  launch_scan_u32_to_u64(b->dp_hist, b->dp_offs, (int64_t)nh, b->dp_scan, s);
  launch_radix_down_pairs(b->dp_keys, b->dp_vals, d_nnz, n, 0, 8, b->dp_offs, b->dp_keys2,
                          reinterpret_cast<uint32_t*>(b->d_items), s);
  k_plan_starts<<<1, 256, 0, s>>>(b->dp_offs, ntiles, d_starts);
  if ((st = ctx_hip(c, hipGetLastError(), "batch plan")) ||
      (st = ctx_hip(c, hipMemcpyAsync(b->pin_starts.p, d_starts, sizeof(uint64_t) * kStarts,
                                      hipMemcpyDeviceToHost, s),
                    "batch plan")) ||
      (st = ctx_hip(c, hipStreamSynchronize(s), "batch plan")))
    return st;
  const uint64_t* sp = static_cast<const uint64_t*>(b->pin_starts.p);
  *nB = (size_t)sp[65];
  *need = (size_t)sp[kHubDigit];
  for (int c2 = 0; c2 <= 64; ++c2) cntA[c2] = (size_t)(sp[65 + (64 - c2) + 1] - sp[65 + (64 - c2)]);
  const size_t nC = (size_t)(sp[kDigits] - sp[kHubDigit]);
  C->clear();
  if (!with_hubs || !nC) return PANTHER_OK;
  const int32_t* hub_idx = b->d_items + sp[kHubDigit];
  if ((st = grow(c, b->dp_hubL, b->dp_hubL_cap, nC, sizeof(uint64_t), "batch plan")) ||
      (st = pinned_ensure(c, b->pin_hubL, sizeof(uint64_t) * nC, "batch plan")) ||
      (st = pinned_ensure(c, b->pin_hubI, sizeof(int32_t) * nC, "batch plan")))
    return st;
  k_plan_hub_lengths<<<(unsigned)((nC + 255) / 256), 256, 0, s>>>(hub_idx, (int64_t)nC, dqlen,
                                                                  b->dp_hubL);
  if ((st = ctx_hip(c, hipGetLastError(), "batch plan")) ||
      (st = ctx_hip(c, hipMemcpyAsync(b->pin_hubL.p, b->dp_hubL, sizeof(uint64_t) * nC,
                                      hipMemcpyDeviceToHost, s),
                    "batch plan")) ||
      (st = ctx_hip(c, hipMemcpyAsync(b->pin_hubI.p, hub_idx, sizeof(int32_t) * nC,
                                      hipMemcpyDeviceToHost, s),
                    "batch plan")) ||
      (st = ctx_hip(c, hipStreamSynchronize(s), "batch plan")))
    return st;
  const uint64_t* hl = static_cast<const uint64_t*>(b->pin_hubL.p);
  const int32_t* hi = static_cast<const int32_t*>(b->pin_hubI.p);
  C->resize(nC);
  for (size_t i = 0; i < nC; ++i) (*C)[i] = {hl[i], hi[i]};
  return PANTHER_OK;
}

// Builds the plan for one configuration.  With `with_hubs` false the hub
// queries are left out (the autotuner times the persistent kernel alone).
// qlen == nullptr: the batch is planned on the device from dqlen.
static int plan(panther_ctx* c, BatchState* b, const BatchConfig& cfg, const int32_t* dq,
                const uint64_t* qlen, const uint64_t* dqlen, int64_t nq, int32_t k, int32_t* d_ids,
                uint32_t* d_counts, int32_t* d_len, float* theta, hipStream_t s, bool with_hubs,
                Plan* out, std::vector<int32_t>* host_items) {
  const Layout lay = layout_for(c, cfg);
  const uint64_t T = (uint64_t)c->T;
  uint64_t LA = (uint64_t)lay.TA / (2 * T);
  uint64_t LB = (uint64_t)lay.TB / (2 * T) / (uint64_t)cfg.tier_b_div;
  if (b->tier_a_override >= 0) LA = std::min(LA, (uint64_t)b->tier_a_override);
  if (b->tier_b_override >= 0) LB = std::min(LB, (uint64_t)b->tier_b_override);
  // the wave-tier sort buffer holds TA/2 keys and the block selection keeps
  // at most kCand keys without radix narrowing; both are covered by the
  // load bound T * L <= table / 2.  The LDS tiers are ordered by
  // power-of-two length class, longest first (enough for load balance):
  // a counting sort over (tier, class) in two passes, written straight
  // into the pinned upload buffer; hubs go exactly longest-first (so that
  // repeated queries of one vertex run side by side and share its rows in
  // the caches), by a stable radix sort on the length.
  // Large batches split both passes over host threads (each thread takes a
  // contiguous range of queries; positions are prefix sums over (tier,
  // class, thread), so the order is the same as one thread's).
  auto cls = [](uint64_t L) { return L ? 64 - __builtin_clzll(L) : 0; };
  std::array<size_t, 65> cntA{};  // tier A items per length class
  size_t nB = 0, need = 0;
  std::vector<std::pair<uint64_t, int32_t>> C;
  int st;
  const bool on_device = qlen == nullptr;
  if (on_device) {
    if ((st = plan_on_device(c, b, dqlen, nq, LA, LB, s, with_hubs, &nB, &need, cntA, &C)))
      return st;
  } else {
    const int nth = nq >= (int64_t)1 << 22 ? 16 : (nq >= (int64_t)1 << 20 ? 8 : 1);
    std::vector<std::array<size_t, 131>> cnt(nth);  // [tier 0: 0..64, tier 1: 65..129, hubs: 130]
    auto range = [&](int t, int64_t& lo, int64_t& hi) {
      lo = nq * t / nth;
      hi = nq * (t + 1) / nth;
    };
    auto count_part = [&](int t) {
      auto& ct = cnt[t];
      ct.fill(0);
      int64_t lo, hi;
      range(t, lo, hi);
      for (int64_t i = lo; i < hi; ++i) {
        const uint64_t L = qlen[i];
        if (L > LB)
          ++ct[130];
        else
          ++ct[(L > LA ? 0 : 65) + cls(L)];  // tier 0: work-group (B), 1: wave (A)
      }
    };
    auto run_parts = [&](auto&& fn) {
      if (nth == 1) {
        fn(0);
        return;
      }
      std::vector<std::thread> th;
      for (int t = 1; t < nth; ++t) th.emplace_back(fn, t);
      fn(0);
      for (auto& x : th) x.join();
    };
    run_parts(count_part);
    // start of each (bucket, thread): buckets in order tier 0 classes 64..0,
    // tier 1 classes 64..0
    std::vector<std::array<size_t, 130>> pos(nth);
    size_t nC = 0;
    for (int tier = 0; tier < 2; ++tier) {
      for (int c2 = 64; c2 >= 0; --c2) {
        const int bk = tier * 65 + c2;
        for (int t = 0; t < nth; ++t) {
          pos[t][bk] = need;
          need += cnt[t][bk];
        }
      }
      if (tier == 0) nB = need;
    }
    for (int t = 0; t < nth; ++t) nC += cnt[t][130];
    for (int c2 = 0; c2 <= 64; ++c2)
      for (int t = 0; t < nth; ++t) cntA[c2] += cnt[t][65 + c2];
    // the pinned staging of the previous plan must have been consumed
    if (b->upload_pending) {
      if ((st = ctx_hip(c, hipEventSynchronize(b->uploaded), "batch plan"))) return st;
      b->upload_pending = false;
    }
    if (need && (st = pinned_ensure(c, b->pin_items, sizeof(int32_t) * need, "batch plan")))
      return st;
    int32_t* items = static_cast<int32_t*>(b->pin_items.p);
    if (with_hubs) C.resize(nC);
    std::vector<size_t> cpos(nth);
    for (int t = 0, run = 0; t < nth; ++t) {
      cpos[t] = run;
      run += (int)cnt[t][130];
    }
    auto scatter_part = [&](int t) {
      auto& pt = pos[t];
      size_t cp = cpos[t];
      int64_t lo, hi;
      range(t, lo, hi);
      for (int64_t i = lo; i < hi; ++i) {
        const uint64_t L = qlen[i];
        if (L > LB) {
          if (with_hubs) C[cp++] = {L, (int32_t)i};
        } else {
          items[pt[(L > LA ? 0 : 65) + cls(L)]++] = (int32_t)i;
        }
      }
    };
    run_parts(scatter_part);
  }
  // tier A phases: class c (lengths below 2^c) runs in groups of G lanes
  // when T * (2^c - 1) fits half of the group's table (kWaveTA * G / 64);
  // the classes are in descending order, so each phase is a range
  auto fits = [&](int c2, int G) {
    return c2 < 32 && T * (((uint64_t)1 << c2) - 1) <= (uint64_t)(kWaveTA * G / kWave / 2);
  };
  size_t nA64 = 0, nA32 = 0, nA16 = 0;
  for (int c2 = 64; c2 >= 0; --c2) {
    const size_t m = cntA[c2];
    if (!fits(c2, 32)) nA64 += m;
    if (!fits(c2, 16)) nA32 += m;
    if (!fits(c2, 8)) nA16 += m;
  }
  // the pinned hub plan of the previous call must have been consumed too
  if (b->upload_pending) {
    if ((st = ctx_hip(c, hipEventSynchronize(b->uploaded), "batch plan"))) return st;
    b->upload_pending = false;
  }
  if (!on_device) sort_hubs_longest_first(C, b->hub_sort_tmp);
  st = plan_hubs(c, b, C, dq, k, cfg.bucket_bias, d_ids, d_counts, d_len, theta, s, &out->hub);
  if (st) return st;
  host_items->clear();
  if (!on_device &&
      (st = grow(c, b->d_items, b->items_cap, std::max<size_t>(need, 1024), sizeof(int32_t),
                 "batch plan")))
    return st;
  if (!b->d_queue) {
    void* p;
    st = ctx_alloc(c, &p, 64, "batch queue");
    if (st) return st;
    b->d_queue = static_cast<uint32_t*>(p);
  }
  if (!on_device && need) {
    st = ctx_hip(c, hipMemcpyAsync(b->d_items, b->pin_items.p, sizeof(int32_t) * need,
                                   hipMemcpyHostToDevice, s),
                 "batch plan upload");
    if (st) return st;
  }
  if (need) {
    if ((st = grow(c, b->d_irec, b->irec_cap, need, sizeof(ItemRec), "batch plan"))) return st;
    k_expand_items<<<(unsigned)((need + 255) / 256), 256, 0, s>>>(b->d_items, (int64_t)need, dq,
                                                                   c->d_inv_ptr, b->d_irec);
    if ((st = ctx_hip(c, hipGetLastError(), "batch plan"))) return st;
  }
  if (!b->uploaded) {
    st = ctx_hip(c, hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming), "batch plan");
    if (st) return st;
  }
  st = ctx_hip(c, hipEventRecord(b->uploaded, s), "batch plan");
  if (st) return st;
  b->upload_pending = true;
  BatchArgs a{};
  a.queries = dq;
  a.itemsB = b->d_irec;
  a.itemsA = b->d_irec + nB;
  a.nB = (int32_t)nB;
  a.nA = (int32_t)(need - nB);
  a.nA64 = (int32_t)nA64;
  a.nA32 = (int32_t)nA32;
  a.nA16 = (int32_t)nA16;
  a.inv_ptr = c->d_inv_ptr;
  a.inv_pid = c->d_inv_pid;
  a.paths = c->d_paths;
  a.queue = b->d_queue;
  a.n = c->n;
  a.k = k;
  a.TB = lay.TB;
  a.out_ids = d_ids;
  a.out_counts = d_counts;
  a.out_len = d_len;
  a.theta = theta;
  a.fR = (float)c->R;
  out->args = a;
  out->run_kernel = need > 0;
  out->stride = c->stride;
  return PANTHER_OK;
}

// Device bytes one query with path list length L adds to a batched call
// of this lane with k <= kmax (an upper bound: per-chunk buffers are sized
// by the largest chunk, and every query is counted whole): its plan entry
// and list length, and for a hub query its staging in row and bucket order,
// bucket counters and maps, winners and tile maps.
BatchSizing batched_sizing(panther_ctx* c, Lane* lane) {
  BatchState* b = state(lane);
  BatchSizing z{};
  z.T = (uint64_t)c->T;
  z.LB = ~0ull;
  z.bucket_bias = 0;
  // before its first call a lane may still pick any configuration
  const std::vector<BatchConfig> cs = b->tuned ? std::vector<BatchConfig>{b->cfg} : config_space(b);
  for (const BatchConfig& cf : cs) {
    const Layout lay = layout_for(c, cf);
    z.LB = std::min<uint64_t>(z.LB, (uint64_t)lay.TB / (2 * z.T) / (uint64_t)cf.tier_b_div);
    z.bucket_bias = std::max(z.bucket_bias, cf.bucket_bias);
  }
  if (b->tier_b_override >= 0) z.LB = std::min(z.LB, (uint64_t)b->tier_b_override);
  z.hub_bits_max = b->hub_bits_max;
  return z;
}

size_t batched_query_bytes(const BatchSizing& z, uint64_t L, int32_t kmax) {
  const uint64_t T = z.T;
  size_t bytes = sizeof(int32_t) + sizeof(uint64_t) + sizeof(ItemRec);
  if (L <= z.LB) return bytes;
  const uint64_t occ = T * L;
  const uint64_t nb = hub_buckets(occ << z.bucket_bias, z.hub_bits_max);
  const uint64_t cand = std::min<uint64_t>((uint64_t)std::max(kmax, kEmitCap) * nb, occ);
  bytes += 2 * sizeof(int32_t) * occ;                                       // staging
  bytes += (3 * sizeof(uint32_t) + 2 * sizeof(uint64_t) + sizeof(int32_t)) * nb;  // buckets
  bytes += scan_temp_bytes((int64_t)nb) + sizeof(uint64_t) * cand + sizeof(uint32_t);
  bytes += sizeof(HubQuery) + sizeof(HubList) +
           sizeof(int32_t) * ((size_t)hub_tiles(L) + hub_stiles(L));
  bytes += sizeof(uint32_t) * ((size_t)hub_stiles(L) * nb);  // per-tile bucket counts
  return bytes;
}

// Device bytes of a batched call's fixed buffers (plan minimum, queue).
size_t batched_fixed_bytes() { return sizeof(int32_t) * 1024 + 64 + sizeof(uint32_t) * 16 + 256; }

// Device bytes the lane's query scratch holds now.
size_t lane_device_bytes(const Lane* lane) {
  size_t t = 0;
  for (const DevBuf* d : {&lane->b_qlen, &lane->b_pool, &lane->b_out, &lane->b_stats, &lane->b_q,
                          &lane->b_qrows, &lane->b_fb, &lane->b_fbw, &lane->b_qsort,
                          &lane->b_qsort_tmp})
    t += d->p ? d->cap : 0;
  const BatchState* b = lane->batch;
  if (!b) return t;
  t += sizeof(int32_t) * b->items_cap + sizeof(ItemRec) * b->irec_cap + (b->d_queue ? 64 : 0);
  t += sizeof(HubQuery) * b->hq_cap + sizeof(int32_t) * (b->occ_cap + b->occB_cap);
  t += sizeof(uint32_t) * (b->bkt_cap + b->bkt_fill_cap + b->redo_cap + b->cand_n_cap);
  t += sizeof(uint64_t) * (b->bkt_start_cap + b->cand_cap + b->bkt_cand0_cap);
  t += sizeof(HubList) * b->hx_cap + b->scan_cap;
  t += sizeof(int32_t) * (b->tile_owner_cap + b->stile_owner_cap + b->bkt_owner_cap);
  t += sizeof(uint32_t) * b->th_cap;
  t += sizeof(uint32_t) * (b->dp_cap + b->dp_keys2_cap + b->dp_vals_cap + b->dp_hist_cap);
  t += sizeof(uint64_t) * (b->dp_offs_cap + b->dp_small_cap + b->dp_hubL_cap) + b->dp_scan_cap;
  return t;
}

int run_batched(panther_ctx* c, Lane* lane, const int32_t* dq, const uint64_t* qlen, int64_t nq,
                int32_t k, int32_t* d_ids, uint32_t* d_counts, int32_t* d_len, float* theta,
                hipStream_t s) {
  BatchState* b = state(lane);
  std::vector<int32_t> items;
  Plan args;
  const uint64_t* dqlen = static_cast<const uint64_t*>(lane->b_qlen.p);
  // configuration: forced, cached, autotuned, or the default
  if (b->forced_block || b->forced_wgs || b->forced_div || b->forced_bias >= 0) {
    BatchConfig f;
    if (b->forced_block) f.block = b->forced_block;
    if (b->forced_wgs) f.wgs_per_cu = b->forced_wgs;
    if (b->forced_div) f.tier_b_div = b->forced_div;
    if (b->forced_bias >= 0) f.bucket_bias = b->forced_bias;
    b->cfg = f;
    b->tuned = true;
  }
  const bool forced = b->forced_block || b->forced_wgs || b->forced_div || b->forced_bias >= 0;
  // the tuned choice is kept per shape class: graph and path count, and the
  // batch size and k rounded to powers of two
  int nq_bucket = 0;
  while ((int64_t(2) << nq_bucket) <= nq) ++nq_bucket;
  int k_bucket = 1;
  while (k_bucket < k) k_bucket <<= 1;
  char key[256];
  snprintf(key, sizeof key, "gfx950:n%d:T%d:R%lld:nq2^%d:k%d:cu%d:f%d", c->n, c->T,
           (long long)c->R, nq_bucket, k_bucket, c->num_cus, theta ? 1 : 0);
  if (b->tuned && !forced && b->tune_key != key) b->tuned = false;
  if (!b->tuned) {
    b->tune_key = key;
    BatchConfig cached;
    if (tune_lookup(b->tune_key, &cached)) {
      b->cfg = cached;
      b->tuned = true;
    } else if (c->autotune && !b->no_tune && nq >= 256) {
      // Results are identical for every configuration by construction; only
      // speed differs.  Stage 1 times the persistent kernel alone on (a
      // prefix of) this batch for each (block, work-groups per CU); stage 2,
      // when the batch has lists near or above the tier B bound and at most
      // kStage2MaxQueries queries, times the whole call for each (tier B
      // divisor, bucket bias).  Each candidate
      // runs once to warm up and is then timed twice (the faster counts).
      // the tuner plans prefixes on the host: a batch planned on the device
      // brings back the lengths of the prefix it times
      const int64_t m = std::min<int64_t>(nq, 16384);
      const uint64_t* tq = qlen;
      if (!tq) {
        int st0 = pinned_ensure(c, lane->h_qlen, sizeof(uint64_t) * (size_t)m, "autotune");
        if (!st0)
          st0 = ctx_hip(c, hipMemcpyAsync(lane->h_qlen.p, dqlen, sizeof(uint64_t) * (size_t)m,
                                          hipMemcpyDeviceToHost, s),
                        "autotune");
        if (!st0) st0 = ctx_hip(c, hipStreamSynchronize(s), "autotune");
        if (st0) return st0;
        tq = static_cast<const uint64_t*>(lane->h_qlen.p);
      }
      hipEvent_t e0, e1;
      int st = ctx_hip(c, hipEventCreate(&e0), "autotune");
      if (st) return st;
      st = ctx_hip(c, hipEventCreate(&e1), "autotune");
      if (st) {
        (void)hipEventDestroy(e0);
        return st;
      }
      auto time_cfg = [&](const BatchConfig& cfg, int64_t m, bool hubs, float* ms_out) -> int {
        int r = plan(c, b, cfg, dq, hubs ? qlen : tq, dqlen, m, k, d_ids, d_counts, d_len, theta,
                     s, hubs, &args, &items);
        if (r) return r;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          (void)hipEventRecord(e0, s);
          if ((r = launch_batched(c, b, cfg, args, s, false))) return r;
          (void)hipEventRecord(e1, s);
          if ((r = ctx_hip(c, hipEventSynchronize(e1), "autotune"))) return r;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) best_ms = std::min(best_ms, ms);
        }
        *ms_out = best_ms;
        return PANTHER_OK;
      };
      BatchConfig best_cfg{};
      float best = 1e30f;
      for (int blk : kBlocks)
        for (int wgs : kWgs) {
          const BatchConfig cfg{blk, wgs, 1, 0};
          float ms = 0.f;
          if (!st) st = time_cfg(cfg, m, false, &ms);
          if (!st && ms < best) {
            best = ms;
            best_cfg = cfg;
          }
        }
      if (!st) {
        const Layout lay = layout_for(c, best_cfg);
        uint64_t LB = (uint64_t)lay.TB / (2 * (uint64_t)c->T);
        if (b->tier_b_override >= 0) LB = std::min(LB, (uint64_t)b->tier_b_override);
        const uint64_t lo = LB / (uint64_t)kTierBDivs[1];
        // (stage 2 replays the whole call twelve times: not for batches so
        // large, such as a feature pass over every vertex, that one call
        // already takes long)
        bool near_hubs = false;
        if (nq <= kStage2MaxQueries)  // (qlen is on the host for such batches)
          for (int64_t i = 0; i < nq && !near_hubs; ++i) near_hubs = qlen[i] > lo;
        if (near_hubs) {
          best = 1e30f;
          const BatchConfig base = best_cfg;
          for (int div : kTierBDivs)
            for (int bias : kBucketBiases) {
              const BatchConfig cfg{base.block, base.wgs_per_cu, div, bias};
              float ms = 0.f;
              if (!st) st = time_cfg(cfg, nq, true, &ms);
              if (!st && ms < best) {
                best = ms;
                best_cfg = cfg;
              }
            }
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (st) return st;
      b->cfg = best_cfg;
      b->tuned = true;
      tune_store(b->tune_key, b->cfg);
    } else {
      b->cfg = BatchConfig{};
      b->tuned = true;
    }
  }
  int st = plan(c, b, b->cfg, dq, qlen, dqlen, nq, k, d_ids, d_counts, d_len, theta, s, true,
                &args, &items);
  if (st) return st;
  // the plan's pinned staging is guarded by b->uploaded; nothing here waits
  return launch_batched(c, b, b->cfg, args, s, true);
}
