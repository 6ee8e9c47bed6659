// Graph preparation (Eq. 3's transition step): CSR validation, per-row
// weight sums W_v, the start set {v : W_v > 0}, and per-row inclusive weight
// prefixes, plus the device-wide exclusive scan used here and by the index.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock)
k_validate(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t n,
           int64_t m, uint32_t* err) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * kBlock;
  uint32_t e = 0;
  for (int64_t v = gid; v < n; v += gsz)
    if (row_ptr[v + 1] < row_ptr[v]) e |= 1u;
  for (int64_t i = gid; i < m; i += gsz) {
    const int32_t c = col[i];
    if (c < 0 || c >= n) e |= 2u;
  }
  if (e) atomicOr(err, e);
}

// Symmetry check of an undirected CSR (Sec. 2, Definition 1: E holds
// unordered pairs, so the entry v->u of weight w is stored in both rows).
// Pass 1 marks the rows whose columns ascend; pass 2 takes one wavefront
// per row and, for every entry (v, u, w), compares how many entries of row v
// read (u, w) with how many of row u read (v, w) -- multi-edges must match
// in number.  Ascending rows are searched by bisection, others scanned.
__global__ void __launch_bounds__(kBlock)
k_rows_sorted(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t n,
              uint8_t* __restrict__ sorted) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t v = wave; v < n; v += nwaves) {
    const int32_t a = row_ptr[v], b = row_ptr[v + 1];
    bool ok = true;
    for (int32_t e = a + 1 + lane; e < b; e += kWave) ok = ok && col[e - 1] <= col[e];
    const bool all = __ballot(!ok) == 0ull;
    if (lane == 0) sorted[v] = all ? 1 : 0;
  }
}

// Entries of row r equal to (t, wt).
__device__ __forceinline__ uint32_t row_matches(const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col,
                                                const uint32_t* __restrict__ w,
                                                const uint8_t* __restrict__ sorted, int32_t r,
                                                int32_t t, uint32_t wt) {
  int32_t lo = row_ptr[r];
  const int32_t hi = row_ptr[r + 1];
  uint32_t c = 0;
  if (sorted[r]) {
    int32_t h = hi;
    while (lo < h) {  // first entry with col >= t
      const int32_t mid = lo + ((h - lo) >> 1);
      if (col[mid] < t)
        lo = mid + 1;
      else
        h = mid;
    }
    for (int32_t e = lo; e < hi && col[e] == t; ++e) c += w[e] == wt ? 1u : 0u;
  } else {
    for (int32_t e = lo; e < hi; ++e) c += (col[e] == t && w[e] == wt) ? 1u : 0u;
  }
  return c;
}

__global__ void __launch_bounds__(kBlock)
k_check_symmetric(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                  const uint32_t* __restrict__ w, const uint8_t* __restrict__ sorted, int32_t n,
                  uint32_t* err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  bool bad = false;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int32_t a = row_ptr[v], b = row_ptr[v + 1];
    for (int32_t e = a + lane; e < b; e += kWave) {
      const int32_t u = col[e];
      const uint32_t wt = w[e];
      if (u == (int32_t)v) continue;  // a self-loop is its own reverse
      if (row_matches(row_ptr, col, w, sorted, (int32_t)v, u, wt) !=
          row_matches(row_ptr, col, w, sorted, u, (int32_t)v, wt))
        bad = true;
    }
  }
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(err, 4u);
}

__global__ void __launch_bounds__(kBlock)
k_rowsum(const int32_t* __restrict__ row_ptr, const uint32_t* __restrict__ w, int32_t n,
         VRec* __restrict__ vrec, unsigned long long* max_w, int32_t* big_rows,
         uint32_t* n_big) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  uint64_t s = 0;
  if (v < n) {
    const int32_t a = row_ptr[v], b = row_ptr[v + 1];
    if (b - a > 256) {
      big_rows[atomicAdd(n_big, 1u)] = v;
      vrec[v] = VRec{a, b - a, 0u, 0u};
    } else {
      for (int32_t e = a; e < b; ++e) s += w[e];
      vrec[v] = VRec{a, b - a, (uint32_t)s, (uint32_t)(s >> 32)};
    }
  }
  s = wave_max(s);
  if ((threadIdx.x & (kWave - 1)) == 0 && s) atomicMax(max_w, (unsigned long long)s);
}

// one wave per long row
__global__ void __launch_bounds__(kBlock)
k_rowsum_big(const int32_t* __restrict__ big_rows, uint32_t n_big, const uint32_t* __restrict__ w,
             VRec* __restrict__ vrec, unsigned long long* max_w) {
  const uint32_t r = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (r >= n_big) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t v = big_rows[r];
  const VRec rec = vrec[v];
  uint64_t s = 0;
  for (int32_t e = rec.start + lane; e < rec.start + rec.deg; e += kWave) s += w[e];
  s = wave_sum(s);
  if (lane == 0) {
    vrec[v].w_lo = (uint32_t)s;
    vrec[v].w_hi = (uint32_t)(s >> 32);
    atomicMax(max_w, (unsigned long long)s);
  }
}

__global__ void __launch_bounds__(kBlock)
k_start_flags(const VRec* __restrict__ vrec, int32_t n, int start_all, uint32_t* flags) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const VRec r = vrec[v];
  flags[v] = (start_all || (r.w_lo | r.w_hi)) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock)
k_start_scatter(const uint32_t* __restrict__ flags, const uint64_t* __restrict__ pos, int32_t n,
                int32_t* __restrict__ vstart) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n && flags[v]) vstart[pos[v]] = v;
}

// Short rows: one thread per row.  Long rows: one wave per row with a
// running carry across 64-entry chunks.
template <typename P>
__global__ void __launch_bounds__(kBlock)
k_prefix_small(const VRec* __restrict__ vrec, const uint32_t* __restrict__ w, int32_t n,
               P* __restrict__ pfx) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const VRec r = vrec[v];
  if (r.deg > 256) return;
  uint64_t s = 0;
  for (int32_t e = r.start; e < r.start + r.deg; ++e) {
    s += w[e];
    pfx[e] = (P)s;
  }
}

template <typename P>
__global__ void __launch_bounds__(kBlock)
k_prefix_big(const VRec* __restrict__ vrec, const uint32_t* __restrict__ w,
             const int32_t* __restrict__ big_rows, uint32_t n_big, P* __restrict__ pfx) {
  const uint32_t r = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (r >= n_big) return;
  const int lane = threadIdx.x & (kWave - 1);
  const VRec rec = vrec[big_rows[r]];
  uint64_t carry = 0;
  for (int32_t base = rec.start; base < rec.start + rec.deg; base += kWave) {
    const int32_t e = base + lane;
    const uint64_t x = e < rec.start + rec.deg ? (uint64_t)w[e] : 0ull;
    const uint64_t inc = wave_inclusive_sum(x);
    if (e < rec.start + rec.deg) pfx[e] = (P)(carry + inc);
    carry += __shfl(inc, kWave - 1, kWave);
  }
}

// ---- walk acceleration (32-bit prefixes): packed edges and guide table ----
// edge[e] = {inclusive weight prefix, column}: one 8-byte load gives both.
__global__ void __launch_bounds__(kBlock)
k_pack_edges(const uint32_t* __restrict__ pfx, const int32_t* __restrict__ col, int64_t m,
             uint2* __restrict__ edge) {
  const int64_t gsz = (int64_t)gridDim.x * kBlock;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m; e += gsz)
    edge[e] = make_uint2(pfx[e], (uint32_t)col[e]);
}

// Guide entry b of a row of degree d: the draws r with floor(r d / 2^64) = b
// are r in [ceil(b 2^64 / d), ceil((b+1) 2^64 / d)); the smallest of them
// gives the smallest u = floor(r W / 2^64), and the first edge with prefix
// > that u is where the selection for any draw of the bucket can start.
// ceil(b 2^64 / d) = b Q + ceil(b Rm / d) with Q = floor(2^64 / d) and
// Rm = 2^64 mod d, all in 64-bit integers.
__device__ __forceinline__ int32_t guide_entry(const uint32_t* __restrict__ pfx, int32_t start,
                                               int32_t deg, uint64_t W, uint64_t b) {
  const uint64_t d = (uint64_t)deg;
  uint64_t Q = ~0ull / d;
  uint64_t Rm = ~0ull - Q * d + 1ull;
  if (Rm == d) {
    Q += 1ull;
    Rm = 0ull;
  }
  const uint64_t rmin = b * Q + (b * Rm + d - 1ull) / d;
  const uint64_t u = __umul64hi(rmin, W);
  int32_t lo = start, hi = start + deg - 1;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)pfx[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kBlock)
k_guide_small(const VRec* __restrict__ vrec, const uint32_t* __restrict__ pfx, int32_t n,
              int32_t* __restrict__ guide) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const VRec r = vrec[v];
  const uint64_t W = (uint64_t)r.w_lo | ((uint64_t)r.w_hi << 32);
  if (r.deg > 256 || r.deg == 0 || W == 0) return;
  for (int32_t b = 0; b < r.deg; ++b) guide[r.start + b] = guide_entry(pfx, r.start, r.deg, W, b);
}

__global__ void __launch_bounds__(kBlock)
k_guide_big(const VRec* __restrict__ vrec, const uint32_t* __restrict__ pfx,
            const int32_t* __restrict__ big_rows, uint32_t n_big, int32_t* __restrict__ guide) {
  const uint32_t r = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (r >= n_big) return;
  const int lane = threadIdx.x & (kWave - 1);
  const VRec rec = vrec[big_rows[r]];
  const uint64_t W = (uint64_t)rec.w_lo | ((uint64_t)rec.w_hi << 32);
  if (W == 0) return;
  for (int32_t b = lane; b < rec.deg; b += kWave)
    guide[rec.start + b] = guide_entry(pfx, rec.start, rec.deg, W, b);
}

// Fat guide record of bucket b (64 bytes, 16 words): the first three
// candidate edges from the guide entry e0 onward, each as {inclusive
// prefix, column, target's row start, target's degree, target's W}, and e0
// itself in word 15.  Candidates past the row end repeat the last edge, whose
// prefix W_v exceeds every draw, so they are never preferred.
__device__ __forceinline__ void fat_record(const VRec* __restrict__ vrec,
                                           const uint32_t* __restrict__ pfx,
                                           const int32_t* __restrict__ col, int32_t start,
                                           int32_t deg, int32_t e0, uint4* __restrict__ out) {
  uint32_t w[16];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int32_t e = e0 + j;
    if (e > start + deg - 1) e = start + deg - 1;
    const int32_t t = col[e];
    const VRec r = vrec[t];
    w[5 * j + 0] = pfx[e];
    w[5 * j + 1] = (uint32_t)t;
    w[5 * j + 2] = (uint32_t)r.start;
    w[5 * j + 3] = (uint32_t)r.deg;
    w[5 * j + 4] = r.w_lo;
  }
  w[15] = (uint32_t)e0;
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

__global__ void __launch_bounds__(kBlock)
k_fat_small(const VRec* __restrict__ vrec, const uint32_t* __restrict__ pfx,
            const int32_t* __restrict__ col, const int32_t* __restrict__ guide, int32_t n,
            uint4* __restrict__ fat) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const VRec r = vrec[v];
  if (r.deg > 256 || r.deg == 0 || (r.w_lo | r.w_hi) == 0) return;
  for (int32_t b = 0; b < r.deg; ++b)
    fat_record(vrec, pfx, col, r.start, r.deg, guide[r.start + b], fat + 4 * (int64_t)(r.start + b));
}

__global__ void __launch_bounds__(kBlock)
k_fat_big(const VRec* __restrict__ vrec, const uint32_t* __restrict__ pfx,
          const int32_t* __restrict__ col, const int32_t* __restrict__ guide,
          const int32_t* __restrict__ big_rows, uint32_t n_big, uint4* __restrict__ fat) {
  const uint32_t rr = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (rr >= n_big) return;
  const int lane = threadIdx.x & (kWave - 1);
  const VRec r = vrec[big_rows[rr]];
  if ((r.w_lo | r.w_hi) == 0) return;
  for (int32_t b = lane; b < r.deg; b += kWave)
    fat_record(vrec, pfx, col, r.start, r.deg, guide[r.start + b], fat + 4 * (int64_t)(r.start + b));
}

// Start records: {vertex, row start, degree, W} of each start-set entry, so
// the walk's first step reads one 16-byte record instead of two lines.
__global__ void __launch_bounds__(kBlock)
k_start_records(const int32_t* __restrict__ vstart, int32_t nstart, const VRec* __restrict__ vrec,
                int4* __restrict__ out) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nstart) return;
  const int32_t v = vstart[i];
  const VRec r = vrec[v];
  out[i] = make_int4(v, r.start, r.deg, (int32_t)r.w_lo);
}

// ---- device-wide exclusive scan (reduce tiles, scan tile sums, apply) ----
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void __launch_bounds__(kBlock)
k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, uint64_t* __restrict__ tile_sums) {
  __shared__ uint64_t red[kBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kBlock + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  s = wave_sum(s);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
    tile_sums[blockIdx.x] = t;
  }
}

// single block: exclusive scan of the tile sums in place; total at [ntiles].
// 256 threads of four sums each: a 1,024-thread block found no room beside
// a persistent kernel on another stream and waited for it to end.
constexpr int kScanPer = 4;
__global__ void __launch_bounds__(kBlock) k_scan_tiles(uint64_t* tile_sums, int64_t ntiles) {
  __shared__ uint64_t s[kBlock / kWave + 1];
  uint64_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += kBlock * kScanPer) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanPer;
    uint64_t x[kScanPer];
    uint64_t loc = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      x[j] = i0 + j < ntiles ? tile_sums[i0 + j] : 0ull;
      loc += x[j];
    }
    uint64_t tot;
    uint64_t run = carry + block_exclusive_sum<kBlock>(loc, s, &tot);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (i0 + j < ntiles) tile_sums[i0 + j] = run;
      run += x[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) tile_sums[ntiles] = carry;
}

__global__ void __launch_bounds__(kBlock)
k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint64_t* __restrict__ tile_sums,
             uint64_t* __restrict__ out) {
  __shared__ uint64_t s[kBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint64_t x[kScanItems];
  uint64_t loc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    x[i] = idx < n ? (uint64_t)in[idx] : 0ull;
    loc += x[i];
  }
  uint64_t tot;
  uint64_t run = tile_sums[blockIdx.x] + block_exclusive_sum<kBlock>(loc, s, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += x[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_sums[gridDim.x];
}

inline unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 30) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (int64_t)cap) g = cap;
  return (unsigned)g;
}

}  // namespace

void launch_validate(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                     uint32_t* err, hipStream_t s) {
  const int64_t work = m > n ? m : n;
  k_validate<<<grid_for(work, kBlock * 8, 65536), kBlock, 0, s>>>(row_ptr, col, n, m, err);
}

void launch_check_symmetric(const int32_t* row_ptr, const int32_t* col, const uint32_t* w,
                            int32_t n, uint8_t* sorted, uint32_t* err, hipStream_t s) {
  const unsigned g = grid_for(n, kBlock / kWave, 65536);
  k_rows_sorted<<<g, kBlock, 0, s>>>(row_ptr, col, n, sorted);
  k_check_symmetric<<<g, kBlock, 0, s>>>(row_ptr, col, w, sorted, n, err);
}

void launch_rowsum(const int32_t* row_ptr, const uint32_t* w, int32_t n, VRec* vrec,
                   uint64_t* max_w, int32_t* big_rows, uint32_t* n_big, hipStream_t s) {
  k_rowsum<<<grid_for(n, kBlock), kBlock, 0, s>>>(row_ptr, w, n, vrec,
                                                  (unsigned long long*)max_w, big_rows, n_big);
}

void launch_rowsum_big(const int32_t* big_rows, uint32_t n_big, const uint32_t* w, VRec* vrec,
                       uint64_t* max_w, hipStream_t s) {
  if (!n_big) return;
  k_rowsum_big<<<grid_for(n_big, kBlock / kWave), kBlock, 0, s>>>(
      big_rows, n_big, w, vrec, (unsigned long long*)max_w);
}

void launch_start_flags(const VRec* vrec, int32_t n, int start_all, uint32_t* flags,
                        hipStream_t s) {
  k_start_flags<<<grid_for(n, kBlock), kBlock, 0, s>>>(vrec, n, start_all, flags);
}

void launch_start_scatter(const uint32_t* flags, const uint64_t* pos, int32_t n, int32_t* vstart,
                          hipStream_t s) {
  k_start_scatter<<<grid_for(n, kBlock), kBlock, 0, s>>>(flags, pos, n, vstart);
}

void launch_prefix32(const VRec* vrec, const uint32_t* w, int32_t n, const int32_t* big_rows,
                     uint32_t n_big, uint32_t* pfx, hipStream_t s) {
  k_prefix_small<uint32_t><<<grid_for(n, kBlock), kBlock, 0, s>>>(vrec, w, n, pfx);
  if (n_big)
    k_prefix_big<uint32_t><<<grid_for(n_big, kBlock / kWave), kBlock, 0, s>>>(vrec, w, big_rows,
                                                                            n_big, pfx);
}

void launch_prefix64(const VRec* vrec, const uint32_t* w, int32_t n, const int32_t* big_rows,
                     uint32_t n_big, uint64_t* pfx, hipStream_t s) {
  k_prefix_small<uint64_t><<<grid_for(n, kBlock), kBlock, 0, s>>>(vrec, w, n, pfx);
  if (n_big)
    k_prefix_big<uint64_t><<<grid_for(n_big, kBlock / kWave), kBlock, 0, s>>>(vrec, w, big_rows,
                                                                            n_big, pfx);
}

void launch_pack_edges(const uint32_t* pfx, const int32_t* col, int64_t m, uint2* edge,
                       hipStream_t s) {
  if (m) k_pack_edges<<<grid_for(m, kBlock * 8, 65536), kBlock, 0, s>>>(pfx, col, m, edge);
}

void launch_guide(const VRec* vrec, const uint32_t* pfx, int32_t n, const int32_t* big_rows,
                  uint32_t n_big, int32_t* guide, hipStream_t s) {
  k_guide_small<<<grid_for(n, kBlock), kBlock, 0, s>>>(vrec, pfx, n, guide);
  if (n_big)
    k_guide_big<<<grid_for(n_big, kBlock / kWave), kBlock, 0, s>>>(vrec, pfx, big_rows, n_big,
                                                                  guide);
}

void launch_fat_guide(const VRec* vrec, const uint32_t* pfx, const int32_t* col,
                      const int32_t* guide, int32_t n, const int32_t* big_rows, uint32_t n_big,
                      uint4* fat, hipStream_t s) {
  k_fat_small<<<grid_for(n, kBlock), kBlock, 0, s>>>(vrec, pfx, col, guide, n, fat);
  if (n_big)
    k_fat_big<<<grid_for(n_big, kBlock / kWave), kBlock, 0, s>>>(vrec, pfx, col, guide, big_rows,
                                                                n_big, fat);
}

void launch_start_records(const int32_t* vstart, int32_t nstart, const VRec* vrec, int4* out,
                          hipStream_t s) {
  k_start_records<<<grid_for(nstart, kBlock), kBlock, 0, s>>>(vstart, nstart, vrec, out);
}

size_t scan_temp_bytes(int64_t n) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  return sizeof(uint64_t) * (size_t)(tiles + 2);
}

void launch_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, void* temp,
                            hipStream_t s) {
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles < 1) tiles = 1;
  uint64_t* ts = static_cast<uint64_t*>(temp);
  k_scan_reduce<<<(unsigned)tiles, kBlock, 0, s>>>(in, n, ts);
  k_scan_tiles<<<1, kBlock, 0, s>>>(ts, tiles);
  k_scan_apply<<<(unsigned)tiles, kBlock, 0, s>>>(in, n, ts, out);
}

}  // namespace panther
