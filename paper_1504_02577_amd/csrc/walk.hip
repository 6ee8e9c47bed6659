// GenerateRandomPath (Algorithm 3): one thread per path.
//
// Step 0 draws the start uniformly from the start set; step t >= 1 moves
// from v along the first CSR entry of v's row whose inclusive weight prefix
// exceeds u = floor(r_t * W_v / 2^64), which selects neighbour j with
// probability w_vj / W_v (Eq. 3).  A weightless row (start-all form only)
// keeps the walk in place.
//
// Rows whose weight sums fit 32 bits use a guide table: bucket
// b = floor(r_t * deg / 2^64) names the first edge e0 any draw of that bucket
// can select.  Its 64-byte record (one aligned line) holds the edges e0,
// e0+1, e0+2 with their inclusive prefixes, targets and the targets' own
// {row start, degree, W}, so the usual step reads one line and already has
// the next vertex's record; only when the draw lies beyond e0+2 does the
// step scan packed {prefix, column} records and load the vertex record.
// The chosen edge is always the first whose prefix exceeds u, as in a
// bisection.
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
         const uint4* __restrict__ fat, const int4* __restrict__ start_rec, int32_t nstart,
         int32_t T, uint64_t R, PhiloxKey key, int32_t* __restrict__ paths) {
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (pid >= R) return;
  int32_t row[S];
  const int4 s0 = start_rec[scale64(draw(key, pid, 0u), (uint64_t)nstart)];
  int32_t v = s0.x;
  row[0] = v;
  VRec cur = VRec{s0.y, s0.z, (uint32_t)s0.w, 0u};
#pragma unroll
  for (int t = 1; t < S; ++t) {
    if (t <= T) {
      const uint64_t r = draw(key, pid, (uint32_t)t);
      const uint32_t W = cur.w_lo;  // w_hi == 0 on this path
      if (W != 0u) {
        const uint32_t u = (uint32_t)scale64(r, (uint64_t)W);
        const uint4* g = fat + 4 * (int64_t)(cur.start + (int32_t)scale64(r, (uint64_t)cur.deg));
        const uint4 g0 = g[0], g1 = g[1], g2 = g[2], g3 = g[3];
        // words: [pfx0 col0 st0 dg0] [W0 pfx1 col1 st1] [dg1 W1 pfx2 col2] [st2 dg2 W2 e0]
        if (u < g0.x) {
          v = (int32_t)g0.y;
          cur = VRec{(int32_t)g0.z, (int32_t)g0.w, g1.x, 0u};
        } else if (u < g1.y) {
          v = (int32_t)g1.z;
          cur = VRec{(int32_t)g1.w, (int32_t)g2.x, g2.y, 0u};
        } else if (u < g2.z) {
          v = (int32_t)g2.w;
          cur = VRec{(int32_t)g3.x, (int32_t)g3.y, g3.z, 0u};
        } else {
          // rare: scan on from the fourth candidate, bisection after kScanMax
          int32_t e = (int32_t)g3.w + 3;
          uint2 x = edge[e];
          int steps = 0;
          while (x.x <= u && steps < kScanMax) {
            ++e;
            x = edge[e];
            ++steps;
          }
          if (x.x <= u) {
            int32_t lo = e + 1, hi = cur.start + cur.deg - 1;
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
          cur = vrec[v];
        }
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

void launch_walk32(int stride, const VRec* vrec, const uint2* edge, const uint4* fat,
                   const int4* start_rec, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                   int32_t* paths, hipStream_t s) {
  const PhiloxKey key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
#define PANTHER_W32(SS) \
  k_walk32<SS><<<grid, kBlock, 0, s>>>(vrec, edge, fat, start_rec, nstart, T, R, key, paths)
  PANTHER_STRIDES(PANTHER_W32)
#undef PANTHER_W32
}

}  // namespace panther
