// Vertex-to-path inverted index (Sec. 3.1; Algorithm 3 "add p_r into P_v").
//
// P_v is a set: a path that visits v several times is listed once.  Build:
// (1) per-vertex list lengths by atomics over the de-duplicated path rows,
// (2) exclusive scan -> inv_ptr, (3) scatter of path ids through per-vertex
// atomic cursors, (4) per-list sort into ascending path id, which makes the
// result independent of the order in which the atomics landed.  Lists of
// length 2..64 are sorted by one wave each (rank by comparison), 65..4096
// by one work-group bitonic sort in LDS, longer ones by 4096-entry chunk
// sorts followed by merge-path passes.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;

template <int S>
__global__ void __launch_bounds__(kBlock)
k_index_count(const int32_t* __restrict__ paths, uint64_t R, uint32_t* __restrict__ cnt) {
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (pid >= R) return;
  int32_t v[S];
  load_row<S>(paths, pid, v);
  dedup_row<S>(v);
#pragma unroll
  for (int i = 0; i < S; ++i)
    if (v[i] >= 0) atomicAdd(&cnt[v[i]], 1u);
}

template <int S>
__global__ void __launch_bounds__(kBlock)
k_index_scatter(const int32_t* __restrict__ paths, uint64_t R,
                unsigned long long* __restrict__ cursor, uint32_t* __restrict__ inv_pid) {
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (pid >= R) return;
  int32_t v[S];
  load_row<S>(paths, pid, v);
  dedup_row<S>(v);
#pragma unroll
  for (int i = 0; i < S; ++i)
    if (v[i] >= 0) inv_pid[atomicAdd(&cursor[v[i]], 1ull)] = (uint32_t)pid;
}

// One wave per vertex.  Lists of length <= 64 are sorted in registers by
// rank: each lane's element moves to the number of smaller elements.
__global__ void __launch_bounds__(kBlock)
k_seg_sort_small(const uint64_t* __restrict__ inv_ptr, int32_t n, uint32_t* __restrict__ inv_pid,
                 int32_t* mid, uint32_t* n_mid, int32_t* big, uint32_t* n_big) {
  const int32_t v = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (v >= n) return;
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t a = inv_ptr[v];
  const uint64_t len = inv_ptr[v + 1] - a;
  if (len <= 1) return;
  if (len > 64) {
    if (lane == 0) {
      if (len <= 4096)
        mid[atomicAdd(n_mid, 1u)] = v;
      else
        big[atomicAdd(n_big, 1u)] = v;
    }
    return;
  }
  const uint32_t x = lane < (int)len ? inv_pid[a + lane] : 0xFFFFFFFFu;
  int rank = 0;
  for (int j = 0; j < (int)len; ++j) {
    const uint32_t y = __shfl(x, j, kWave);
    rank += (y < x) ? 1 : 0;
  }
  if (lane < (int)len) inv_pid[a + rank] = x;
}

constexpr int kMidCap = 4096;

__global__ void __launch_bounds__(kBlock)
k_seg_sort_mid(const uint64_t* __restrict__ inv_ptr, const int32_t* __restrict__ mid,
               uint32_t* __restrict__ inv_pid) {
  __shared__ uint32_t s[kMidCap];
  const int32_t v = mid[blockIdx.x];
  const uint64_t a = inv_ptr[v];
  const int len = (int)(inv_ptr[v + 1] - a);
  const int P = next_pow2(len);
  for (int i = threadIdx.x; i < P; i += kBlock) s[i] = i < len ? inv_pid[a + i] : 0xFFFFFFFFu;
  __syncthreads();
  block_bitonic_asc<kBlock>(s, P);
  for (int i = threadIdx.x; i < len; i += kBlock) inv_pid[a + i] = s[i];
}

// Big lists, step 1: sort each 4096-entry chunk in place.
__global__ void __launch_bounds__(kBlock)
k_seg_chunk_sort(const SegBlock* __restrict__ blocks, uint32_t* __restrict__ data) {
  __shared__ uint32_t s[kMidCap];
  const SegBlock b = blocks[blockIdx.x];
  const uint64_t base = b.start + b.off;
  const uint32_t rem = b.len - b.off;
  const int cnt = (int)(rem < (uint32_t)kMidCap ? rem : (uint32_t)kMidCap);
  const int P = next_pow2(cnt < 2 ? 2 : cnt);
  for (int i = threadIdx.x; i < P; i += kBlock) s[i] = i < cnt ? data[base + i] : 0xFFFFFFFFu;
  __syncthreads();
  block_bitonic_asc<kBlock>(s, P);
  for (int i = threadIdx.x; i < cnt; i += kBlock) data[base + i] = s[i];
}

// Big lists, step 2: merge sorted runs of `width` pairwise.  Each block
// writes 4096 outputs (16 per thread) of one merged pair; each thread finds
// its start on the merge path by bisection.
constexpr int kMergeItems = 16;
constexpr int kMergeTile = kBlock * kMergeItems;

__global__ void __launch_bounds__(kBlock)
k_seg_merge(const SegBlock* __restrict__ blocks, uint32_t width, const uint32_t* __restrict__ src,
            uint32_t* __restrict__ dst) {
  const SegBlock b = blocks[blockIdx.x];
  const uint64_t w2 = 2ull * width;
  const uint64_t pair0 = (b.off / w2) * w2;  // start of the pair within the list
  const uint64_t alen = (pair0 + width < b.len ? pair0 + width : b.len) - pair0;
  const uint64_t bend = pair0 + w2 < b.len ? pair0 + w2 : b.len;
  const uint64_t blen = bend > pair0 + alen ? bend - pair0 - alen : 0;
  const uint32_t* A = src + b.start + pair0;
  const uint32_t* B = A + alen;
  const uint64_t total = alen + blen;
  uint64_t diag = (b.off - pair0) + (uint64_t)threadIdx.x * kMergeItems;
  if (diag >= total) return;
  // merge path: i from A, diag - i from B
  uint64_t lo = diag > blen ? diag - blen : 0;
  uint64_t hi = diag < alen ? diag : alen;
  while (lo < hi) {
    const uint64_t m = (lo + hi) >> 1;
    if (A[m] <= B[diag - 1 - m])
      lo = m + 1;
    else
      hi = m;
  }
  uint64_t i = lo, j = diag - lo;
  uint32_t* out = dst + b.start + pair0 + diag;
  for (int t = 0; t < kMergeItems && diag + t < total; ++t) {
    bool takeA;
    if (i >= alen)
      takeA = false;
    else if (j >= blen)
      takeA = true;
    else
      takeA = A[i] <= B[j];
    out[t] = takeA ? A[i++] : B[j++];
  }
}

__global__ void __launch_bounds__(kBlock)
k_seg_copy(const SegBlock* __restrict__ blocks, const uint32_t* __restrict__ src,
           uint32_t* __restrict__ dst) {
  const SegBlock b = blocks[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kMergeTile && b.off + i < b.len; i += kBlock)
    dst[b.start + b.off + i] = src[b.start + b.off + i];
}

}  // namespace

void launch_index_count(int stride, const int32_t* paths, uint64_t R, uint32_t* cnt,
                        hipStream_t s) {
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
  switch (stride) {
    case 4: k_index_count<4><<<grid, kBlock, 0, s>>>(paths, R, cnt); break;
    case 8: k_index_count<8><<<grid, kBlock, 0, s>>>(paths, R, cnt); break;
    case 16: k_index_count<16><<<grid, kBlock, 0, s>>>(paths, R, cnt); break;
    case 32: k_index_count<32><<<grid, kBlock, 0, s>>>(paths, R, cnt); break;
    default: k_index_count<64><<<grid, kBlock, 0, s>>>(paths, R, cnt); break;
  }
}

void launch_index_scatter(int stride, const int32_t* paths, uint64_t R,
                          unsigned long long* cursor, uint32_t* inv_pid, hipStream_t s) {
  const unsigned grid = (unsigned)((R + kBlock - 1) / kBlock);
  switch (stride) {
    case 4: k_index_scatter<4><<<grid, kBlock, 0, s>>>(paths, R, cursor, inv_pid); break;
    case 8: k_index_scatter<8><<<grid, kBlock, 0, s>>>(paths, R, cursor, inv_pid); break;
    case 16: k_index_scatter<16><<<grid, kBlock, 0, s>>>(paths, R, cursor, inv_pid); break;
    case 32: k_index_scatter<32><<<grid, kBlock, 0, s>>>(paths, R, cursor, inv_pid); break;
    default: k_index_scatter<64><<<grid, kBlock, 0, s>>>(paths, R, cursor, inv_pid); break;
  }
}

void launch_seg_sort_small(const uint64_t* inv_ptr, int32_t n, uint32_t* inv_pid, int32_t* mid,
                           uint32_t* n_mid, int32_t* big, uint32_t* n_big, hipStream_t s) {
  const unsigned grid = (unsigned)((n + kBlock / kWave - 1) / (kBlock / kWave));
  k_seg_sort_small<<<grid, kBlock, 0, s>>>(inv_ptr, n, inv_pid, mid, n_mid, big, n_big);
}

void launch_seg_sort_mid(const uint64_t* inv_ptr, const int32_t* mid, uint32_t n_mid,
                         uint32_t* inv_pid, hipStream_t s) {
  if (n_mid) k_seg_sort_mid<<<n_mid, kBlock, 0, s>>>(inv_ptr, mid, inv_pid);
}

void launch_seg_chunk_sort(const SegBlock* blocks, uint32_t nblocks, uint32_t* data,
                           hipStream_t s) {
  if (nblocks) k_seg_chunk_sort<<<nblocks, kBlock, 0, s>>>(blocks, data);
}

void launch_seg_merge(const SegBlock* blocks, uint32_t nblocks, uint32_t width,
                      const uint32_t* src, uint32_t* dst, hipStream_t s) {
  if (nblocks) k_seg_merge<<<nblocks, kBlock, 0, s>>>(blocks, width, src, dst);
}

void launch_seg_copy(const SegBlock* blocks, uint32_t nblocks, const uint32_t* src,
                     uint32_t* dst, hipStream_t s) {
  if (nblocks) k_seg_copy<<<nblocks, kBlock, 0, s>>>(blocks, src, dst);
}

}  // namespace panther
