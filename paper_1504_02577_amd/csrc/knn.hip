// Panther++ nearest neighbours in double precision (Sec. 3.3): for each
// query q, the k vertices v != q of smallest squared Euclidean distance
// between feature rows, ties by id.  The kd-tree of the paper indexes this
// same exact search; here every row is scanned (brute force).
//
// Arithmetic per pair: d2 = 0; for d in 0..D-1: delta = (double)theta_q[d]
// - (double)theta_v[d]; d2 = fma(delta, delta, d2) -- one fused multiply-add
// per coordinate in coordinate order.
//
// The cross-graph form takes the query rows from another graph's features
// and ranks every row of this one (no row is the query itself).
//
// A work-group takes QT queries (their rows in LDS as doubles) and streams
// all n rows, one row per thread per round.  Each query keeps a candidate
// buffer in LDS with a threshold (the kp-th best (d2, id) kept so far):
// candidates below it are appended; at the end of a round any buffer with
// more than kp entries is bitonic-sorted by one wavefront and cut back to
// kp, which tightens the threshold.  A round adds at most 256 entries, so a
// 512-entry buffer never overflows for kp <= 256.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace panther {

namespace {

constexpr int kBlock = 256;
constexpr int kBuf = 512;

__device__ __forceinline__ void wave_sync_knn() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bool pair_less(double a, int32_t va, double b, int32_t vb) {
  return a < b || (a == b && va < vb);
}

// Ascending bitonic sort of cnt (d2, id) pairs by one wavefront.
__device__ void wave_sort_pairs(double* d, int32_t* v, int cnt) {
  const int lane = threadIdx.x & (kWave - 1);
  int P = 2;
  while (P < cnt) P <<= 1;
  for (int i = cnt + lane; i < P; i += kWave) {
    d[i] = INFINITY;
    v[i] = 0x7FFFFFFF;
  }
  wave_sync_knn();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (P >> 1); i += kWave) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const double a = d[lo], b = d[hi];
        const int32_t x = v[lo], y = v[hi];
        if (pair_less(b, y, a, x) == asc) {
          d[lo] = b;
          d[hi] = a;
          v[lo] = y;
          v[hi] = x;
        }
      }
      wave_sync_knn();
    }
  }
}

template <int QT>
__global__ void __launch_bounds__(kBlock)
k_knn_fp64(const float* __restrict__ theta, int32_t n, int32_t D,
           const float* __restrict__ qtheta, int32_t exclude_self,
           const int32_t* __restrict__ queries, int64_t nq, int32_t k, int32_t kp,
           int32_t* __restrict__ out_ids, double* __restrict__ out_dist) {
  extern __shared__ __align__(16) char lds[];
  double* qv = reinterpret_cast<double*>(lds);      // [QT][D]
  double* bd = qv + QT * D;                          // [QT][kBuf]
  int32_t* bv = reinterpret_cast<int32_t*>(bd + QT * kBuf);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(bv + QT * kBuf);
  double* tau_d = reinterpret_cast<double*>(cnt + QT + (QT & 1));
  int32_t* tau_v = reinterpret_cast<int32_t*>(tau_d + QT);
  int32_t* qid = tau_v + QT;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t q0 = (int64_t)blockIdx.x * QT;
  for (int i = threadIdx.x; i < QT; i += kBlock) {
    qid[i] = (q0 + i < nq) ? queries[q0 + i] : -1;
    cnt[i] = 0u;
    tau_d[i] = INFINITY;
    tau_v[i] = 0x7FFFFFFF;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < QT * D; i += kBlock) {
    const int32_t q = qid[i / D];
    qv[i] = q >= 0 ? (double)qtheta[(int64_t)q * D + (i % D)] : 0.0;
  }
  __syncthreads();
  for (int64_t base = 0; base < n; base += kBlock) {
    const int64_t v = base + threadIdx.x;
    double acc[QT];
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[q] = 0.0;
    if (v < n) {
      const float* row = theta + v * D;
      for (int d = 0; d < D; ++d) {
        const double x = (double)row[d];
#pragma unroll
        for (int q = 0; q < QT; ++q) {
          const double delta = qv[q * D + d] - x;
          acc[q] = fma(delta, delta, acc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < QT; ++q) {
      const int32_t me = qid[q];
      if (v < n && me >= 0 && (!exclude_self || (int32_t)v != me) &&
          pair_less(acc[q], (int32_t)v, tau_d[q], tau_v[q])) {
        const uint32_t pos = atomicAdd(&cnt[q], 1u);
        bd[q * kBuf + pos] = acc[q];
        bv[q * kBuf + pos] = (int32_t)v;
      }
    }
    __syncthreads();
    for (int q = wid; q < QT; q += kBlock / kWave) {
      const int c = (int)cnt[q];
      if (c > kp) {
        wave_sort_pairs(bd + q * kBuf, bv + q * kBuf, c);
        if (lane == 0) {
          cnt[q] = (uint32_t)kp;
          tau_d[q] = bd[q * kBuf + kp - 1];
          tau_v[q] = bv[q * kBuf + kp - 1];
        }
      }
    }
    __syncthreads();
  }
  for (int q = wid; q < QT; q += kBlock / kWave) {
    if (qid[q] < 0) continue;
    const int c = (int)cnt[q];
    wave_sort_pairs(bd + q * kBuf, bv + q * kBuf, c);
    const int64_t qi = q0 + q;
    for (int j = lane; j < k; j += kWave) {
      const bool ok = j < c;
      out_ids[qi * k + j] = ok ? bv[q * kBuf + j] : -1;
      out_dist[qi * k + j] = ok ? sqrt(bd[q * kBuf + j]) : INFINITY;
    }
    wave_sync_knn();
  }
}

}  // namespace

size_t knn_fp64_lds(int D) {
  constexpr int QT = 16;
  return sizeof(double) * QT * D + (sizeof(double) + sizeof(int32_t)) * QT * kBuf +
         sizeof(uint32_t) * (QT + 1) + (sizeof(double) + 2 * sizeof(int32_t)) * QT + 64;
}

// qtheta: the queries' feature rows (theta itself for one graph, the other
// graph's for the cross-graph form, which excludes no row).
int launch_knn_fp64(const float* theta, int32_t n, int32_t D, const float* qtheta,
                    bool exclude_self, const int32_t* queries, int64_t nq, int32_t k,
                    int32_t* out_ids, double* out_dist, hipStream_t s) {
  constexpr int QT = 16;
  int kp = 1;
  while (kp < k) kp <<= 1;
  const size_t lds = knn_fp64_lds(D);
  hipError_t e = hipFuncSetAttribute((const void*)k_knn_fp64<QT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return (int)e;
  const unsigned grid = (unsigned)((nq + QT - 1) / QT);
  if (grid)
    k_knn_fp64<QT><<<grid, kBlock, lds, s>>>(theta, n, D, qtheta, exclude_self ? 1 : 0, queries,
                                              nq, k, kp, out_ids, out_dist);
  return (int)hipGetLastError();
}

}  // namespace panther
