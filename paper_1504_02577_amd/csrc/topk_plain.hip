// Panther query, plain form (Algorithm 1 + the top-k step), one kernel
// launch per query.
//
// Every thread takes one path id of P_q, loads the path row, drops repeated
// vertices and q itself, and increments a dense per-vertex counter in global
// memory; the first increment of a vertex appends it to a touched list
// (wave-aggregated).  The last work-group to finish (atomic ticket) selects
// the k largest (count, -id) keys over the touched list, writes them, and
// clears the counters it used, so the dense array is zero again for the
// next launch.
#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The query id is read from device memory (*qp).  An id outside [0, n)
// writes a padded row with out_len = -1 and touches no counter.
template <int S>
__global__ void __launch_bounds__(kBlock)
k_topk_plain(const int32_t* __restrict__ qp, int32_t n, const uint64_t* __restrict__ inv_ptr,
             const uint32_t* __restrict__ inv_pid, const int32_t* __restrict__ paths,
             uint32_t* cnt, int32_t* touched, uint32_t* ctl, int32_t k,
             int32_t* __restrict__ out_ids, uint32_t* __restrict__ out_counts,
             int32_t* __restrict__ out_len) {
  __shared__ SelectSmem sm;
  __shared__ uint32_t s_last;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t q = *qp;
  if (q < 0 || q >= n) {
    if (blockIdx.x == 0) {
      for (int j = threadIdx.x; j < k; j += kBlock) {
        out_ids[j] = -1;
        out_counts[j] = 0u;
      }
      if (threadIdx.x == 0) *out_len = -1;
    }
    return;
  }
  const uint64_t a = inv_ptr[q];
  const uint64_t L = inv_ptr[q + 1] - a;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < L;
       base += (uint64_t)gridDim.x * kBlock) {
    const uint64_t idx = base + threadIdx.x;
    int32_t v[S];
    if (idx < L) {
      load_row<S>(paths, inv_pid[a + idx], v);
      dedup_row<S>(v);
    } else {
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = -1;
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const bool want = v[i] >= 0 && v[i] != q;
      const uint32_t old = want ? atomicAdd(&cnt[v[i]], 1u) : 1u;
      const bool fresh = want && old == 0u;
      const uint64_t mask = __ballot(fresh);
      if (mask) {
        uint32_t wbase = 0;
        if (lane == 0) wbase = atomicAdd(&ctl[0], (uint32_t)__popcll(mask));
        wbase = __shfl(wbase, 0, kWave);
        if (fresh) touched[wbase + __popcll(mask & ((1ull << lane) - 1ull))] = v[i];
      }
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&ctl[1], 1u) == gridDim.x - 1) ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int nt = (int)ld_agent(&ctl[0]);
  auto key = [&](int i) {
    const int32_t v = ld_agent(&touched[i]);
    return rank_key(ld_agent(&cnt[v]), v);
  };
  const int m = block_select_topk<kBlock>(key, nt, k, sm);
  for (int j = threadIdx.x; j < k; j += kBlock) {
    const bool ok = j < m;
    out_ids[j] = ok ? key_vertex(sm.out[j]) : -1;
    out_counts[j] = ok ? key_count(sm.out[j]) : 0u;
  }
  if (threadIdx.x == 0) *out_len = m;
  __syncthreads();
  for (int i = threadIdx.x; i < nt; i += kBlock) cnt[ld_agent(&touched[i])] = 0u;
  if (threadIdx.x == 0) {
    ctl[0] = 0u;
    ctl[1] = 0u;
  }
}

__global__ void k_query_lengths(const uint64_t* __restrict__ inv_ptr,
                                const int32_t* __restrict__ queries, int64_t nq,
                                uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < nq) {
    const int32_t q = queries[i];
    out[i] = inv_ptr[q + 1] - inv_ptr[q];
  }
}

}  // namespace

namespace {
__global__ void k_iota_ids(int32_t* out, int32_t n) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = i;
}
}  // namespace

void launch_iota(int32_t* out, int32_t n, hipStream_t s) {
  k_iota_ids<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n);
}

namespace {
__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0u;
}
}  // namespace

void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  k_zero_u32<<<(unsigned)g, 256, 0, s>>>(p, n);
}

void launch_query_lengths(const uint64_t* inv_ptr, const int32_t* queries, int64_t nq,
                          uint64_t* out, hipStream_t s) {
  if (nq > 0)
    k_query_lengths<<<(unsigned)((nq + kBlock - 1) / kBlock), kBlock, 0, s>>>(inv_ptr, queries, nq,
                                                                            out);
}

void launch_topk_plain(int stride, const int32_t* qp, int32_t n, const uint64_t* inv_ptr,
                       const uint32_t* inv_pid, const int32_t* paths, uint64_t list_len,
                       TopkScratch sc, int32_t k, int32_t* out_ids, uint32_t* out_counts,
                       int32_t* out_len, hipStream_t s) {
  uint64_t g = (list_len + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  const unsigned grid = (unsigned)g;
#define PANTHER_LAUNCH(SS)                                                                    \
  k_topk_plain<SS><<<grid, kBlock, 0, s>>>(qp, n, inv_ptr, inv_pid, paths, sc.cnt,            \
                                           sc.touched, sc.ctl, k, out_ids, out_counts, out_len)
  switch (stride) {
    case 4: PANTHER_LAUNCH(4); break;
    case 8: PANTHER_LAUNCH(8); break;
    case 16: PANTHER_LAUNCH(16); break;
    case 32: PANTHER_LAUNCH(32); break;
    default: PANTHER_LAUNCH(64); break;
  }
#undef PANTHER_LAUNCH
}

}  // namespace panther
