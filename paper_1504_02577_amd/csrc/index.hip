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
// The tile lives in registers (thread t holds items j * 256 + t, so each
// wavefront holds whole 64-item chunks).  The in-tile rank comes from those
// chunks: a wave matches digits across its lanes with one ballot per digit
// bit, chunk histograms (LDS) are scanned per digit, and the rank is chunk
// prefix + lanes below with the same digit.
// No atomics touch global memory, so the order of equal vertices is the
// path-id order of the input and the index is deterministic.
// ---------------------------------------------------------------------------
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kTileItems = 4096;
constexpr int kChunks = kTileItems / kWave;

// Work-group i of a grid of g runs on XCD i % 8 (round-robin dispatch).
// Tile order for the down-sweeps: each XCD takes a contiguous range of
// tiles, so the runs that neighbouring tiles write for one digit (adjacent
// in the output) meet in the same L2 and leave it as whole lines.
__device__ __forceinline__ uint64_t xcd_tile(uint32_t i, uint32_t g) {
  const uint32_t x = i % 8u, j = i / 8u;
  const uint32_t per = g / 8u, rem = g % 8u;
  return (uint64_t)x * per + (x < rem ? x : rem) + j;
}

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift, int bits) {
  return (key >> shift) & ((1u << bits) - 1u);
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_radix_up_paths(const int32_t* __restrict__ paths, uint64_t R, int ppt, int shift, int bits,
                 uint64_t ntiles, uint32_t* __restrict__ hist) {
  // a histogram needs no order: digits straight from the de-duplicated rows
  __shared__ uint32_t s_hist[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kBlock) s_hist[d] = 0u;
  __syncthreads();
  // tiles in the down-sweeps' XCD order, so that the counts of neighbouring
  // tiles (adjacent in the digit-major table) leave one L2 as whole lines
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t p0 = tile * (uint64_t)ppt;
  // RG rows in flight per thread before their digits are counted
  constexpr int RG = S <= 8 ? 4 : (S <= 16 ? 2 : 1);
  for (int r0 = 0; r0 < ppt; r0 += RG * kBlock) {
    int32_t v[RG][S];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int r = r0 + g * kBlock + (int)threadIdx.x;
      const uint64_t pid = p0 + r;
      if (r < ppt && pid < R) {
        load_row<S>(paths, pid, v[g]);
      } else {
#pragma unroll
        for (int i = 0; i < S; ++i) v[g][i] = -1;
      }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      dedup_row<S>(v[g]);
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (v[g][i] >= 0) atomicAdd(&s_hist[digit_of((uint32_t)v[g][i], shift, bits)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kBlock) hist[(uint64_t)d * ntiles + tile] = s_hist[d];
}

// LDS of a down-sweep: the tile's pairs (pass 1 stages them here), then the
// chunk histograms, then the tile reordered by digit.
struct RankSmem {
  union {
    uint16_t chunk[kChunks][kRadix];
    struct {
      uint32_t key[kTileItems];
      uint32_t val[kTileItems];
    } tile;
  } u;
  uint32_t lstart[kRadix];  // first position of digit d in the reordered tile
  uint64_t gbase[kRadix];   // global position of that item
  uint32_t scan[kBlock / kWave + 1];
};
static_assert(kBlock == kRadix, "one digit per thread in the digit scans");

// Ranks a tile held in registers (thread t holds items j * 256 + t) stably
// by digit, reorders it by digit in LDS, and writes each digit's run from
// offset[digit][tile] on, consecutive threads on consecutive addresses.
__device__ __forceinline__ void rank_scatter_regs(const uint32_t (&k)[16], const uint32_t (&v)[16],
                                                  int n, int shift, int bits, RankSmem& sm,
                                                  const uint64_t* __restrict__ offsets,
                                                  uint64_t ntiles, uint64_t tile,
                                                  uint32_t* __restrict__ key_out,
                                                  uint32_t* __restrict__ val_out) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint16_t (*chunk)[kRadix] = sm.u.chunk;
  uint32_t rk[16];
  {
    uint32_t* z = reinterpret_cast<uint32_t*>(&chunk[0][0]);
    for (int i = threadIdx.x; i < kChunks * kRadix / 2; i += kBlock) z[i] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = j * kBlock + threadIdx.x;
    const int c = j * (kBlock / kWave) + wid;
    const bool live = i < n;
    const uint32_t d = live ? digit_of(k[j], shift, bits) : 0u;
    uint64_t same = __ballot(live);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint64_t m = __ballot(live && ((d >> b) & 1u));
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint64_t below = same & ((1ull << lane) - 1ull);
    rk[j] = (uint32_t)__popcll(below);
    if (live && below == 0) chunk[c][d] = (uint16_t)__popcll(same);
  }
  __syncthreads();
  // digit d = thread d: chunk prefix (rank base of each chunk inside the
  // tile), then the digit starts of the reordered tile by a block scan
  const int nchunks = (n + kWave - 1) / kWave;
  {
    const int d = threadIdx.x;
    uint32_t dtot = 0;
#pragma unroll 8
    for (int c = 0; c < nchunks; ++c) {
      const uint32_t x = chunk[c][d];
      chunk[c][d] = (uint16_t)dtot;
      dtot += x;
    }
    uint32_t ttot;
    const uint32_t ls = block_exclusive_sum<kBlock>(dtot, sm.scan, &ttot);
    sm.lstart[d] = ls;
    sm.gbase[d] = offsets[(uint64_t)d * ntiles + tile] - ls;
  }
  __syncthreads();
  uint32_t lp[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = j * kBlock + threadIdx.x;
    lp[j] = 0u;
    if (i < n) {
      const uint32_t d = digit_of(k[j], shift, bits);
      const int c = j * (kBlock / kWave) + wid;
      lp[j] = sm.lstart[d] + chunk[c][d] + rk[j];
    }
  }
  __syncthreads();  // the chunk table is dead from here; its LDS holds the tile
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (j * kBlock + (int)threadIdx.x < n) {
      sm.u.tile.key[lp[j]] = k[j];
      sm.u.tile.val[lp[j]] = v[j];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const uint32_t key = sm.u.tile.key[i];
    const uint64_t pos = sm.gbase[digit_of(key, shift, bits)] + (uint64_t)i;
    key_out[pos] = key;
    val_out[pos] = sm.u.tile.val[i];
  }
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_radix_down_paths(const int32_t* __restrict__ paths, uint64_t R, int ppt, int shift, int bits,
                   uint64_t ntiles, const uint64_t* __restrict__ offsets,
                   uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
  // the compacted (vertex, path id) pairs are staged in path-id order in
  // the tile region, then moved to registers
  __shared__ RankSmem sm;
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t p0 = tile * ppt;
  // thread t takes rows [t * rpt, t * rpt + rpt) of the tile, all loaded
  // before any is used; one block scan orders the pairs by path id
  constexpr int RMAX = S <= 32 ? 32 / S : 1;
  const int rpt = (ppt + kBlock - 1) / kBlock;  // <= RMAX for every T with this S
  int32_t v[RMAX][S];
  uint32_t cnt = 0;
#pragma unroll
  for (int g = 0; g < RMAX; ++g) {
    const int r = (int)threadIdx.x * rpt + g;
    const uint64_t pid = p0 + r;
    if (g < rpt && r < ppt && pid < R) {
      load_row<S>(paths, pid, v[g]);
    } else {
#pragma unroll
      for (int i = 0; i < S; ++i) v[g][i] = -1;
    }
  }
#pragma unroll
  for (int g = 0; g < RMAX; ++g) {
    dedup_row<S>(v[g]);
#pragma unroll
    for (int i = 0; i < S; ++i) cnt += v[g][i] >= 0 ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t o = block_exclusive_sum<kBlock>(cnt, sm.scan, &tot);
#pragma unroll
  for (int g = 0; g < RMAX; ++g) {
    const uint32_t pid = (uint32_t)(p0 + (uint64_t)((int)threadIdx.x * rpt + g));
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (v[g][i] >= 0) {
        sm.u.tile.key[o] = (uint32_t)v[g][i];
        sm.u.tile.val[o] = pid;
        ++o;
      }
  }
  const int base = (int)tot;
  __syncthreads();
  const int n = base;
  uint32_t k[16], vv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = j * kBlock + threadIdx.x;
    k[j] = i < n ? sm.u.tile.key[i] : 0u;
    vv[j] = i < n ? sm.u.tile.val[i] : 0u;
  }
  __syncthreads();
  rank_scatter_regs(k, vv, n, shift, bits, sm, offsets, ntiles, tile, key_out, val_out);
}

__global__ void __launch_bounds__(kBlock)
k_radix_up_pairs(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ nnz_dev,
                 int shift, int bits, uint64_t ntiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_hist[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kBlock) s_hist[d] = 0u;
  __syncthreads();
  const uint64_t nnz = *nnz_dev;  // tiles past it count nothing
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);  // as in k_radix_up_paths
  const uint64_t a = tile * kTileItems;
  // all 16 keys of the thread are loaded before any is counted
  uint32_t k[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint64_t i = a + (uint64_t)j * kBlock + threadIdx.x;
    k[j] = i < nnz ? keys[i] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (k[j] != 0xFFFFFFFFu) atomicAdd(&s_hist[digit_of(k[j], shift, bits)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kBlock) hist[(uint64_t)d * ntiles + tile] = s_hist[d];
}

// Passes >= 2: the tile of 4096 consecutive pairs goes straight to registers.
__global__ void __launch_bounds__(kBlock)
k_radix_down_pairs(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                   const uint64_t* __restrict__ nnz_dev, int shift, int bits, uint64_t ntiles,
                   const uint64_t* __restrict__ offsets, uint32_t* __restrict__ key_out,
                   uint32_t* __restrict__ val_out) {
  __shared__ RankSmem sm;
  const uint64_t nnz = *nnz_dev;
  const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t a = tile * kTileItems;
  if (a >= nnz) return;  // a tile past the pairs: nothing to move
  const int n = (int)((nnz - a) < (uint64_t)kTileItems ? (nnz - a) : (uint64_t)kTileItems);
  uint32_t k[16], v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = j * kBlock + threadIdx.x;
    k[j] = i < n ? keys[a + i] : 0u;
    v[j] = i < n ? vals[a + i] : 0u;
  }
  rank_scatter_regs(k, v, n, shift, bits, sm, offsets, ntiles, tile, key_out, val_out);
}

__global__ void k_copy_u64(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// inv_ptr from the sorted vertex keys: position i opens the lists of every
// vertex in (key[i-1], key[i]], and nnz those after the last key.  Thread t
// takes keys [4t, 4t + 4) with one 16-byte load.
__global__ void __launch_bounds__(kBlock)
k_list_bounds(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ nnz_dev, int32_t n,
              uint64_t* __restrict__ inv_ptr) {
  const uint64_t nnz = *nnz_dev;
  const uint64_t i0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
  if (i0 > nnz) return;
  uint32_t k[4];
  if (i0 + 4 <= nnz) {
    const uint4 x = *reinterpret_cast<const uint4*>(keys + i0);
    k[0] = x.x;
    k[1] = x.y;
    k[2] = x.z;
    k[3] = x.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = i0 + j < nnz ? keys[i0 + j] : (uint32_t)n;
  }
  int64_t kp = i0 == 0 ? -1 : (int64_t)keys[i0 - 1];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t i = i0 + j;
    if (i > nnz) break;
    const int64_t kc = i == nnz ? (int64_t)n : (int64_t)k[j];
    for (int64_t v = kp + 1; v <= kc; ++v) inv_ptr[v] = i;
    kp = kc;
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

void launch_radix_up_pairs(const uint32_t* keys, const uint64_t* nnz_dev, uint64_t nnz_cap,
                           int shift, int bits, uint32_t* hist, hipStream_t s) {
  const uint64_t nt = radix_tiles_pairs(nnz_cap);
  k_radix_up_pairs<<<(unsigned)nt, kBlock, 0, s>>>(keys, nnz_dev, shift, bits, nt, hist);
}

void launch_radix_down_pairs(const uint32_t* keys, const uint32_t* vals, const uint64_t* nnz_dev,
                             uint64_t nnz_cap, int shift, int bits, const uint64_t* offsets,
                             uint32_t* key_out, uint32_t* val_out, hipStream_t s) {
  const uint64_t nt = radix_tiles_pairs(nnz_cap);
  k_radix_down_pairs<<<(unsigned)nt, kBlock, 0, s>>>(keys, vals, nnz_dev, shift, bits, nt, offsets,
                                                      key_out, val_out);
}

void launch_copy_u64(const uint64_t* src, uint64_t* dst, hipStream_t s) {
  k_copy_u64<<<1, 64, 0, s>>>(src, dst);
}

void launch_list_bounds(const uint32_t* keys, const uint64_t* nnz_dev, uint64_t nnz_cap, int32_t n,
                        uint64_t* inv_ptr, hipStream_t s) {
  const uint64_t g = (nnz_cap / 4 + 1 + kBlock - 1) / kBlock;
  k_list_bounds<<<(unsigned)g, kBlock, 0, s>>>(keys, nnz_dev, n, inv_ptr);
}

}  // namespace panther
