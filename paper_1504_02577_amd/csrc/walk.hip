// GenerateRandomPath (Algorithm 3): one thread per path.
//
// Step 0 draws the start uniformly from the start set; step t >= 1 moves
// from v along the first CSR entry of v's row whose inclusive weight prefix
// exceeds u = floor(r_t * W_v / 2^64), which selects neighbour j with
// probability w_vj / W_v (Eq. 3).  A weightless row (start-all form only)
// keeps the walk in place.
//
// Memory per step: one 16-byte vertex record (row start, degree, W_v), a
// bisection over the row's prefix (ceil(log2 deg) 4- or 8-byte probes) and
// one 4-byte column read; the T+1 vertices are written once per path as
// S/4 16-byte stores.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;

template <typename P>
__device__ __forceinline__ int32_t upper_bound_row(const P* __restrict__ pfx, int32_t lo,
                                                   int32_t hi, uint64_t u) {
  // first e in [lo, hi] with pfx[e] > u; pfx[hi] = W_v > u guarantees one
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)pfx[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

template <int S, typename P>
__global__ void __launch_bounds__(kBlock)
k_walk(const VRec* __restrict__ vrec, const P* __restrict__ pfx, const int32_t* __restrict__ col,
       const int32_t* __restrict__ vstart, int32_t nstart, int32_t T, uint64_t R, PhiloxKey key,
       int32_t* __restrict__ paths) {
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
        const int32_t e = upper_bound_row(pfx, rec.start, rec.start + rec.deg - 1, u);
        v = col[e];
      }
      row[t] = v;
    } else {
      row[t] = -1;
    }
  }
  int4* out = reinterpret_cast<int4*>(paths + pid * (uint64_t)S);
#pragma unroll
  for (int i = 0; i < S / 4; ++i)
    out[i] = make_int4(row[4 * i], row[4 * i + 1], row[4 * i + 2], row[4 * i + 3]);
}

template <int S>
void walk_s(bool pfx64, const VRec* vrec, const void* pfx, const int32_t* col,
            const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, PhiloxKey key,
            int32_t* paths, hipStream_t s) {
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
  if (pfx64)
    k_walk<S, uint64_t><<<grid, kBlock, 0, s>>>(vrec, static_cast<const uint64_t*>(pfx), col,
                                                vstart, nstart, T, R, key, paths);
  else
    k_walk<S, uint32_t><<<grid, kBlock, 0, s>>>(vrec, static_cast<const uint32_t*>(pfx), col,
                                                vstart, nstart, T, R, key, paths);
}

}  // namespace

void launch_walk(int stride, bool pfx64, const VRec* vrec, const void* pfx, const int32_t* col,
                 const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                 int32_t* paths, hipStream_t s) {
  const PhiloxKey key{(uint32_t)seed, (uint32_t)(seed >> 32)};
  switch (stride) {
    case 4: walk_s<4>(pfx64, vrec, pfx, col, vstart, nstart, T, R, key, paths, s); break;
    case 8: walk_s<8>(pfx64, vrec, pfx, col, vstart, nstart, T, R, key, paths, s); break;
    case 16: walk_s<16>(pfx64, vrec, pfx, col, vstart, nstart, T, R, key, paths, s); break;
    case 32: walk_s<32>(pfx64, vrec, pfx, col, vstart, nstart, T, R, key, paths, s); break;
    default: walk_s<64>(pfx64, vrec, pfx, col, vstart, nstart, T, R, key, paths, s); break;
  }
}

}  // namespace panther
