// GenerateRandomPath (Algorithm 3): one thread per path.
//
// Step 0 draws the start uniformly from the start set; step t >= 1 moves
// from v along the first CSR entry of v's row whose inclusive weight prefix
// exceeds u = floor(r_t * W_v / 2^64), which selects neighbour j with
// probability w_vj / W_v (Eq. 3).  A weightless row (start-all form only)
// keeps the walk in place.
//
// Rows whose weight sums fit 32 bits use a guide table: bucket
// b = floor(r_t * deg / 2^64) names the first edge any draw of that bucket
// can select, and a short forward scan over packed {prefix, column} records
// (8 bytes, eight to a 64-byte line) finds the edge -- the same edge as a
// bisection, in about one cache line instead of log2(deg).  Per step: one
// 16-byte vertex record, one 4-byte guide entry, and the scanned records.
// Rows with 64-bit sums use the bisection over separate prefix and column
// arrays.  Each path's T+1 vertices are written once as 16-byte stores.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;
constexpr int kScanMax = 8;  // forward steps before falling back to bisection

template <int S>
__device__ __forceinline__ void store_row(int32_t* __restrict__ paths, uint64_t pid,
                                          const int32_t (&row)[S]) {
  int4* out = reinterpret_cast<int4*>(paths + pid * (uint64_t)S);
#pragma unroll
  for (int i = 0; i < S / 4; ++i)
    out[i] = make_int4(row[4 * i], row[4 * i + 1], row[4 * i + 2], row[4 * i + 3]);
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_walk32(const VRec* __restrict__ vrec, const uint2* __restrict__ edge,
         const int32_t* __restrict__ guide, const int32_t* __restrict__ vstart, int32_t nstart,
         int32_t T, uint64_t R, PhiloxKey key, int32_t* __restrict__ paths) {
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (pid >= R) return;
  int32_t row[S];
  int32_t v = vstart[scale64(draw(key, pid, 0u), (uint64_t)nstart)];
  row[0] = v;
#pragma unroll
  for (int t = 1; t < S; ++t) {
    if (t <= T) {
      const uint64_t r = draw(key, pid, (uint32_t)t);
      const VRec rec = vrec[v];
      const uint32_t W = rec.w_lo;  // w_hi == 0 on this path
      if (W != 0u) {
        const uint32_t u = (uint32_t)scale64(r, (uint64_t)W);
        int32_t e = guide[rec.start + (int32_t)scale64(r, (uint64_t)rec.deg)];
        uint2 x = edge[e];
        int steps = 0;
        while (x.x <= u && steps < kScanMax) {
          ++e;
          x = edge[e];
          ++steps;
        }
        if (x.x <= u) {
          // rare: bisection over the rest of the row
          int32_t lo = e + 1, hi = rec.start + rec.deg - 1;
          while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (edge[mid].x > u)
              hi = mid;
            else
              lo = mid + 1;
          }
          x = edge[lo];
        }
        v = (int32_t)x.y;
      }
      row[t] = v;
    } else {
      row[t] = -1;
    }
  }
  store_row<S>(paths, pid, row);
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_walk64(const VRec* __restrict__ vrec, const uint64_t* __restrict__ pfx,
         const int32_t* __restrict__ col, const int32_t* __restrict__ vstart, int32_t nstart,
         int32_t T, uint64_t R, PhiloxKey key, int32_t* __restrict__ paths) {
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (pid >= R) return;
  int32_t row[S];
  int32_t v = vstart[scale64(draw(key, pid, 0u), (uint64_t)nstart)];
  row[0] = v;
#pragma unroll
  for (int t = 1; t < S; ++t) {
    if (t <= T) {
      const uint64_t r = draw(key, pid, (uint32_t)t);
      const VRec rec = vrec[v];
      const uint64_t W = (uint64_t)rec.w_lo | ((uint64_t)rec.w_hi << 32);
      if (W != 0) {
        const uint64_t u = scale64(r, W);
        int32_t lo = rec.start, hi = rec.start + rec.deg - 1;
        while (lo < hi) {
          const int32_t mid = lo + ((hi - lo) >> 1);
          if (pfx[mid] > u)
            hi = mid;
          else
            lo = mid + 1;
        }
        v = col[lo];
      }
      row[t] = v;
    } else {
      row[t] = -1;
    }
  }
  store_row<S>(paths, pid, row);
}

}  // namespace

#define PANTHER_STRIDES(MACRO) \
  switch (stride) {            \
    case 4: MACRO(4); break;   \
    case 8: MACRO(8); break;   \
    case 16: MACRO(16); break; \
    case 32: MACRO(32); break; \
    default: MACRO(64); break; \
  }

void launch_walk64(int stride, const VRec* vrec, const uint64_t* pfx, const int32_t* col,
                   const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                   int32_t* paths, hipStream_t s) {
  const PhiloxKey key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
#define PANTHER_W64(SS) \
  k_walk64<SS><<<grid, kBlock, 0, s>>>(vrec, pfx, col, vstart, nstart, T, R, key, paths)
  PANTHER_STRIDES(PANTHER_W64)
#undef PANTHER_W64
}

void launch_walk32(int stride, const VRec* vrec, const uint2* edge, const int32_t* guide,
                   const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                   int32_t* paths, hipStream_t s) {
  const PhiloxKey key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
#define PANTHER_W32(SS) \
  k_walk32<SS><<<grid, kBlock, 0, s>>>(vrec, edge, guide, vstart, nstart, T, R, key, paths)
  PANTHER_STRIDES(PANTHER_W32)
#undef PANTHER_W32
}

}  // namespace panther
