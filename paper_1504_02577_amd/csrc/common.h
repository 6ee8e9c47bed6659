// Device-side building blocks shared by the Panther kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace panther {

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of the
// 4x32 Philox S-box; multipliers and Weyl increments as published.
// Counter layout for the draw of path `pid`, step `t`: (t, 0, pid lo, pid hi);
// key (seed lo, seed hi); the 64-bit word is x0 | x1 << 32.
// ---------------------------------------------------------------------------
struct PhiloxKey {
  uint32_t k0, k1;
};

__device__ __forceinline__ uint64_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, PhiloxKey key) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
    const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
    const uint32_t n0 = hiB ^ c1 ^ k0;
    const uint32_t n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return (uint64_t)c0 | ((uint64_t)c1 << 32);
}

__device__ __forceinline__ uint64_t draw(PhiloxKey key, uint64_t pid, uint32_t step) {
  return philox_word(step, 0u, (uint32_t)pid, (uint32_t)(pid >> 32), key);
}

// floor(r * n / 2^64)
__device__ __forceinline__ uint64_t scale64(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// ---------------------------------------------------------------------------
// Paths are stored row-major with a padded stride S (a power of two >= T+1);
// slots T+1..S-1 hold -1.  `unique_row` loads a row and replaces every
// repeated vertex (and the padding) by -1, keeping first occurrences.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ void load_row(const int32_t* __restrict__ paths, uint64_t pid,
                                         int32_t (&v)[S]) {
  const int4* p = reinterpret_cast<const int4*>(paths + pid * (uint64_t)S);
#pragma unroll
  for (int i = 0; i < S / 4; ++i) {
    int4 x = p[i];
    v[4 * i + 0] = x.x;
    v[4 * i + 1] = x.y;
    v[4 * i + 2] = x.z;
    v[4 * i + 3] = x.w;
  }
}

template <int S>
__device__ __forceinline__ void dedup_row(int32_t (&v)[S]) {
  int32_t u[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    bool first = v[i] >= 0;
#pragma unroll
    for (int j = 0; j < i; ++j) first = first && (v[j] != v[i]);
    u[i] = first ? v[i] : -1;
  }
#pragma unroll
  for (int i = 0; i < S; ++i) v[i] = u[i];
}

// ---------------------------------------------------------------------------
// Wave / block scans.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    T y = __shfl_xor(x, off, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// Exclusive block scan; returns the block total through *total.  `s` must
// hold BLOCK / 64 elements.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_sum(T x, T* s, T* total) {
  constexpr int kW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  T inc = wave_inclusive_sum(x);
  if (lane == kWave - 1) s[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    T w = lane < kW ? s[lane] : T(0);
    T wi = wave_inclusive_sum(w);
    if (lane < kW) s[lane] = wi - w;
    if (lane == kW - 1) s[kW] = wi;
  }
  __syncthreads();
  T res = s[wid] + inc - x;
  *total = s[kW];
  __syncthreads();
  return res;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_max(T x, T* s) {
  constexpr int kW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  x = wave_max(x);
  if (lane == 0) s[wid] = x;
  __syncthreads();
  T r = s[0];
#pragma unroll
  for (int i = 1; i < kW; ++i) r = s[i] > r ? s[i] : r;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Bitonic sort of P (power of two) keys in LDS, descending.
// ---------------------------------------------------------------------------
template <int BLOCK, typename K>
__device__ __forceinline__ void block_bitonic_desc(K* s, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += BLOCK) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool desc = (lo & size) == 0;
        K a = s[lo], b = s[hi];
        if ((a < b) == desc) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

template <int BLOCK, typename K>
__device__ __forceinline__ void block_bitonic_asc(K* s, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += BLOCK) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        K a = s[lo], b = s[hi];
        if ((a > b) == asc) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

__host__ __device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Ranking key of a candidate: larger is better; count descending, then
// vertex id ascending.  Distinct for distinct vertices; 0 never occurs for
// a candidate with count >= 1.
__device__ __forceinline__ uint64_t rank_key(uint32_t count, int32_t v) {
  return ((uint64_t)count << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)v);
}
__device__ __forceinline__ int32_t key_vertex(uint64_t key) {
  return (int32_t)(0xFFFFFFFFu - (uint32_t)key);
}
__device__ __forceinline__ uint32_t key_count(uint64_t key) { return (uint32_t)(key >> 32); }

// ---------------------------------------------------------------------------
// Block-wide selection of the k largest of n distinct non-zero 64-bit keys,
// produced on demand by key(i), i in [0, n).  Small sets are sorted whole in
// LDS.  Larger sets are narrowed by 11-bit radix histograms (most significant
// digit first) until the class straddling the k-th key fits in LDS; the keys
// above that class are certainly selected.  The result (min(k, n) keys,
// descending) is left in s_out.  LDS: s_cand[kCand], s_hist[kHist],
// s_out[kOutCap], s_misc[8].
// ---------------------------------------------------------------------------
constexpr int kCand = 2048;
constexpr int kOutCap = 1024;
constexpr int kHistBits = 11;
constexpr int kHist = 1 << kHistBits;

struct SelectSmem {
  uint64_t cand[kCand];
  uint64_t out[kOutCap];
  uint32_t hist[kHist];
  uint64_t red[32];
  uint32_t misc[8];
};

template <int BLOCK, typename KeyFn>
__device__ int block_select_topk(KeyFn key, int n, int k, SelectSmem& sm) {
  const int tid = threadIdx.x;
  if (n <= kCand) {
    const int P = next_pow2(n < 2 ? 2 : n);
    for (int i = tid; i < P; i += BLOCK) sm.cand[i] = i < n ? key(i) : 0ull;
    __syncthreads();
    block_bitonic_desc<BLOCK>(sm.cand, P);
    const int m = n < k ? n : k;
    for (int i = tid; i < m; i += BLOCK) sm.out[i] = sm.cand[i];
    __syncthreads();
    return m;
  }
  // --- radix narrowing ---
  uint64_t mx = 0;
  for (int i = tid; i < n; i += BLOCK) {
    uint64_t x = key(i);
    mx = x > mx ? x : mx;
  }
  mx = block_max<BLOCK>(mx, sm.red);
  int shift = 64 - __clzll(mx);  // every key < 2^shift
  uint64_t prefix = 0;           // selected class: key >> shift == prefix
  int need = k;
  uint32_t cls = (uint32_t)n;
  while (shift > 0) {
    const int dbits = shift < kHistBits ? shift : kHistBits;
    const int nsh = shift - dbits;
    const uint32_t nb = 1u << dbits;
    for (int i = tid; i < (int)nb; i += BLOCK) sm.hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += BLOCK) {
      uint64_t x = key(i);
      if ((shift >= 64 ? 0ull : (x >> shift)) == prefix)
        atomicAdd(&sm.hist[(uint32_t)(x >> nsh) & (nb - 1)], 1u);
    }
    __syncthreads();
    // the digit d holding the need-th largest key: fewer than `need` keys
    // of the class lie in digits above d, at least `need` in d and above.
    // Each thread takes a run of digits in descending order; a block scan
    // gives the count above its run, and the one thread whose run holds the
    // crossing records it (the class holds >= need keys, so it exists)
    {
      const int per = ((int)nb + BLOCK - 1) / BLOCK;
      uint64_t loc = 0;
      for (int i = 0; i < per; ++i) {
        const int pos = tid * per + i;
        if (pos < (int)nb) loc += sm.hist[nb - 1 - pos];
      }
      uint64_t tot;
      uint64_t above = block_exclusive_sum<BLOCK>(loc, sm.red, &tot);
      for (int i = 0; i < per; ++i) {
        const int pos = tid * per + i;
        if (pos >= (int)nb) break;
        const uint32_t h = sm.hist[nb - 1 - pos];
        if (above < (uint64_t)need && above + h >= (uint64_t)need) {
          sm.misc[0] = nb - 1 - pos;
          sm.misc[1] = (uint32_t)above;
          sm.misc[2] = h;
        }
        above += h;
      }
    }
    __syncthreads();
    const uint32_t d = sm.misc[0];
    need -= (int)sm.misc[1];
    cls = sm.misc[2];
    prefix = (prefix << dbits) | d;
    shift = nsh;
    __syncthreads();
    if (cls <= (uint32_t)kCand) break;
  }
  // collect: keys above the class are selected; the class is sorted whole
  if (tid == 0) {
    sm.misc[3] = 0;
    sm.misc[4] = 0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += BLOCK) {
    uint64_t x = key(i);
    uint64_t hi = shift >= 64 ? 0ull : (x >> shift);
    if (hi > prefix) {
      uint32_t p = atomicAdd(&sm.misc[3], 1u);
      if (p < (uint32_t)kOutCap) sm.out[p] = x;
    } else if (hi == prefix) {
      uint32_t p = atomicAdd(&sm.misc[4], 1u);
      if (p < (uint32_t)kCand) sm.cand[p] = x;
    }
  }
  __syncthreads();
  // keys are distinct, so these stay within the buffers; clamp regardless
  const int ndef = (int)(sm.misc[3] < (uint32_t)kOutCap ? sm.misc[3] : (uint32_t)kOutCap);
  const int ncls = (int)(sm.misc[4] < (uint32_t)kCand ? sm.misc[4] : (uint32_t)kCand);
  const int P = next_pow2(ncls < 2 ? 2 : ncls);
  for (int i = ncls + tid; i < P; i += BLOCK) sm.cand[i] = 0ull;
  __syncthreads();
  block_bitonic_desc<BLOCK>(sm.cand, P);
  for (int i = tid; i < need; i += BLOCK) sm.out[ndef + i] = sm.cand[i];
  __syncthreads();
  const int m = ndef + need;  // == k
  const int P2 = next_pow2(m < 2 ? 2 : m);
  for (int i = m + tid; i < P2; i += BLOCK) sm.out[i] = 0ull;
  __syncthreads();
  block_bitonic_desc<BLOCK>(sm.out, P2);
  return m;
}

}  // namespace panther
