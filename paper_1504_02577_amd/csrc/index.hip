// Vertex-to-path inverted index (Sec. 3.1; Algorithm 3 "add p_r into P_v").
//
// P_v is a set: a path that visits v several times is listed once, and the
// lists hold path ids in ascending order.  The (vertex, path id) pairs of the
// de-duplicated path rows are sorted by vertex with a stable radix sort, so
// equal vertices keep path-id order; list offsets come from the boundaries
// of the sorted keys.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Stable LSD radix sort of the (vertex, path id) pairs by vertex.
//
// Pass 1 reads the path rows directly: a tile is `ppt` consecutive paths;
// their distinct vertices become pairs in path-id order (compacted in LDS).
// Later passes read tiles of 4096 consecutive pairs.  Each pass has an
// up-sweep (per-tile digit histogram), a device-wide exclusive scan of the
// histograms in digit-major order, and a down-sweep that ranks every item
// stably inside its tile and scatters it to
//   offset[digit][tile] + (same-digit items before it in the tile).
// The in-tile rank comes from 64-item chunks: a wave matches digits across
// its lanes with one ballot per digit bit, chunk histograms are scanned per
// digit, and the rank is chunk prefix + lanes below with the same digit.
// No atomics touch global memory, so the order of equal vertices is the
// path-id order of the input and the index is deterministic.
// ---------------------------------------------------------------------------
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kTileItems = 4096;
constexpr int kChunks = kTileItems / kWave;

struct RadixSmem {
  uint32_t key[kTileItems];
  uint32_t val[kTileItems];
  uint16_t chunk[kChunks][kRadix];  // chunk histograms, then exclusive prefixes
  uint8_t rank[kTileItems];
  uint32_t scan[kBlock / kWave + 1];
  uint32_t n;
};

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift, int bits) {
  return (key >> shift) & ((1u << bits) - 1u);
}

// Loads the distinct vertices of the tile's paths into sm.key/sm.val in
// path-id order; returns the item count.
template <int S>
__device__ int load_tile_from_paths(const int32_t* __restrict__ paths, uint64_t R, uint64_t p0,
                                    int ppt, RadixSmem& sm) {
  int base = 0;
  for (int r0 = 0; r0 < ppt; r0 += kBlock) {
    const uint64_t pid = p0 + r0 + threadIdx.x;
    int32_t v[S];
    const bool live = (r0 + (int)threadIdx.x < ppt) && pid < R;
    if (live) {
      load_row<S>(paths, pid, v);
      dedup_row<S>(v);
    } else {
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = -1;
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < S; ++i) cnt += v[i] >= 0 ? 1u : 0u;
    uint32_t tot;
    uint32_t off = block_exclusive_sum<kBlock>(cnt, sm.scan, &tot);
    uint32_t o = (uint32_t)base + off;
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (v[i] >= 0) {
        sm.key[o] = (uint32_t)v[i];
        sm.val[o] = (uint32_t)pid;
        ++o;
      }
    base += (int)tot;
  }
  __syncthreads();
  return base;
}

__device__ void tile_histogram(const RadixSmem& sm, int n, int shift, int bits, uint32_t* hist,
                               uint32_t* s_hist) {
  for (int d = threadIdx.x; d < kRadix; d += kBlock) s_hist[d] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) atomicAdd(&s_hist[digit_of(sm.key[i], shift, bits)], 1u);
  __syncthreads();
}

// In-tile stable ranks (chunk prefix + in-chunk rank), then the scatter.
__device__ void rank_and_scatter(RadixSmem& sm, int n, int shift, int bits,
                                 const uint64_t* __restrict__ offsets, uint64_t ntiles,
                                 uint64_t tile, uint32_t* __restrict__ key_out,
                                 uint32_t* __restrict__ val_out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nchunks = (n + kWave - 1) / kWave;
  for (int i = threadIdx.x; i < kChunks * kRadix; i += kBlock)
    (&sm.chunk[0][0])[i] = 0;
  __syncthreads();
  for (int c = wid; c < nchunks; c += kBlock / kWave) {
    const int i = c * kWave + lane;
    const bool live = i < n;
    const uint32_t d = live ? digit_of(sm.key[i], shift, bits) : 0xFFFFu;
    uint64_t same = __ballot(live);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint64_t m = __ballot(live && ((d >> b) & 1u));
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    if (live) {
      const uint64_t below = same & ((1ull << lane) - 1ull);
      sm.rank[i] = (uint8_t)__popcll(below);
      if (below == 0) sm.chunk[c][d] = (uint16_t)__popcll(same);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kBlock) {
    uint32_t run = 0;
    for (int c = 0; c < nchunks; ++c) {
      const uint32_t x = sm.chunk[c][d];
      sm.chunk[c][d] = (uint16_t)run;
      run += x;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const uint32_t key = sm.key[i];
    const uint32_t d = digit_of(key, shift, bits);
    const uint64_t pos = offsets[(uint64_t)d * ntiles + tile] + sm.chunk[i / kWave][d] + sm.rank[i];
    if (key_out) key_out[pos] = key;
    val_out[pos] = sm.val[i];
  }
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_radix_up_paths(const int32_t* __restrict__ paths, uint64_t R, int ppt, int shift, int bits,
                 uint64_t ntiles, uint32_t* __restrict__ hist) {
  __shared__ RadixSmem sm;
  __shared__ uint32_t s_hist[kRadix];
  const int n = load_tile_from_paths<S>(paths, R, (uint64_t)blockIdx.x * ppt, ppt, sm);
  tile_histogram(sm, n, shift, bits, hist, s_hist);
  for (int d = threadIdx.x; d < kRadix; d += kBlock) hist[(uint64_t)d * ntiles + blockIdx.x] = s_hist[d];
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_radix_down_paths(const int32_t* __restrict__ paths, uint64_t R, int ppt, int shift, int bits,
                   uint64_t ntiles, const uint64_t* __restrict__ offsets,
                   uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
  __shared__ RadixSmem sm;
  const int n = load_tile_from_paths<S>(paths, R, (uint64_t)blockIdx.x * ppt, ppt, sm);
  rank_and_scatter(sm, n, shift, bits, offsets, ntiles, blockIdx.x, key_out, val_out);
}

__device__ int load_tile_pairs(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                               uint64_t nnz, uint64_t tile, RadixSmem& sm, bool with_vals) {
  const uint64_t a = tile * kTileItems;
  const int n = (int)((nnz - a) < (uint64_t)kTileItems ? (nnz - a) : (uint64_t)kTileItems);
  for (int i = threadIdx.x; i < n; i += kBlock) {
    sm.key[i] = keys[a + i];
    if (with_vals) sm.val[i] = vals[a + i];
  }
  __syncthreads();
  return n;
}

__global__ void __launch_bounds__(kBlock)
k_radix_up_pairs(const uint32_t* __restrict__ keys, uint64_t nnz, int shift, int bits,
                 uint64_t ntiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_hist[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kBlock) s_hist[d] = 0u;
  __syncthreads();
  const uint64_t a = (uint64_t)blockIdx.x * kTileItems;
  for (uint64_t i = a + threadIdx.x; i < a + kTileItems && i < nnz; i += kBlock)
    atomicAdd(&s_hist[digit_of(keys[i], shift, bits)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kBlock) hist[(uint64_t)d * ntiles + blockIdx.x] = s_hist[d];
}

__global__ void __launch_bounds__(kBlock)
k_radix_down_pairs(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                   uint64_t nnz, int shift, int bits, uint64_t ntiles,
                   const uint64_t* __restrict__ offsets, uint32_t* __restrict__ key_out,
                   uint32_t* __restrict__ val_out) {
  __shared__ RadixSmem sm;
  const int n = load_tile_pairs(keys, vals, nnz, blockIdx.x, sm, true);
  rank_and_scatter(sm, n, shift, bits, offsets, ntiles, blockIdx.x, key_out, val_out);
}

// inv_ptr from the sorted vertex keys: position i opens the lists of every
// vertex in (key[i-1], key[i]].
__global__ void __launch_bounds__(kBlock)
k_list_bounds(const uint32_t* __restrict__ keys, uint64_t nnz, int32_t n,
              uint64_t* __restrict__ inv_ptr) {
  const uint64_t gsz = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i <= nnz; i += gsz) {
    const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
    const int64_t kc = i == nnz ? (int64_t)n : (int64_t)keys[i];
    for (int64_t v = kp + 1; v <= kc; ++v) inv_ptr[v] = i;
  }
}

}  // namespace

uint64_t radix_tiles_paths(uint64_t R, int T) {
  const int ppt = kTileItems / (T + 1);
  return (R + ppt - 1) / ppt;
}

uint64_t radix_tiles_pairs(uint64_t nnz) { return (nnz + kTileItems - 1) / kTileItems; }

void launch_radix_up_paths(int stride, const int32_t* paths, uint64_t R, int T, int shift,
                           int bits, uint32_t* hist, hipStream_t s) {
  const int ppt = kTileItems / (T + 1);
  const uint64_t nt = radix_tiles_paths(R, T);
#define PANTHER_UP(SS) \
  k_radix_up_paths<SS><<<(unsigned)nt, kBlock, 0, s>>>(paths, R, ppt, shift, bits, nt, hist)
  switch (stride) {
    case 4: PANTHER_UP(4); break;
    case 8: PANTHER_UP(8); break;
    case 16: PANTHER_UP(16); break;
    case 32: PANTHER_UP(32); break;
    default: PANTHER_UP(64); break;
  }
#undef PANTHER_UP
}

void launch_radix_down_paths(int stride, const int32_t* paths, uint64_t R, int T, int shift,
                             int bits, const uint64_t* offsets, uint32_t* key_out,
                             uint32_t* val_out, hipStream_t s) {
  const int ppt = kTileItems / (T + 1);
  const uint64_t nt = radix_tiles_paths(R, T);
#define PANTHER_DOWN(SS)                                                                   \
  k_radix_down_paths<SS><<<(unsigned)nt, kBlock, 0, s>>>(paths, R, ppt, shift, bits, nt, \
                                                         offsets, key_out, val_out)
  switch (stride) {
    case 4: PANTHER_DOWN(4); break;
    case 8: PANTHER_DOWN(8); break;
    case 16: PANTHER_DOWN(16); break;
    case 32: PANTHER_DOWN(32); break;
    default: PANTHER_DOWN(64); break;
  }
#undef PANTHER_DOWN
}

void launch_radix_up_pairs(const uint32_t* keys, uint64_t nnz, int shift, int bits,
                           uint32_t* hist, hipStream_t s) {
  const uint64_t nt = radix_tiles_pairs(nnz);
  k_radix_up_pairs<<<(unsigned)nt, kBlock, 0, s>>>(keys, nnz, shift, bits, nt, hist);
}

void launch_radix_down_pairs(const uint32_t* keys, const uint32_t* vals, uint64_t nnz, int shift,
                             int bits, const uint64_t* offsets, uint32_t* key_out,
                             uint32_t* val_out, hipStream_t s) {
  const uint64_t nt = radix_tiles_pairs(nnz);
  k_radix_down_pairs<<<(unsigned)nt, kBlock, 0, s>>>(keys, vals, nnz, shift, bits, nt, offsets,
                                                      key_out, val_out);
}

void launch_list_bounds(const uint32_t* keys, uint64_t nnz, int32_t n, uint64_t* inv_ptr,
                        hipStream_t s) {
  uint64_t g = (nnz + 1 + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  k_list_bounds<<<(unsigned)g, kBlock, 0, s>>>(keys, nnz, n, inv_ptr);
}

}  // namespace panther
