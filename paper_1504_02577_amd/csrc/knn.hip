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
#include <algorithm>
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
           const int32_t* __restrict__ queries, const int32_t* __restrict__ rows, int64_t nq,
           int32_t k, int32_t kp,
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
    qid[i] = (q0 + i < nq) ? queries[rows ? rows[q0 + i] : q0 + i] : -1;
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
    const int64_t qi = rows ? (int64_t)rows[q0 + q] : q0 + q;
    for (int j = lane; j < k; j += kWave) {
      const bool ok = j < c;
      out_ids[qi * k + j] = ok ? bv[q * kBuf + j] : -1;
      out_dist[qi * k + j] = ok ? sqrt(bd[q * kBuf + j]) : INFINITY;
    }
    wave_sync_knn();
  }
}

constexpr int kSelCap = 4096;

// Norm band of each listed query over a norm-ordered copy of the database
// (rows of norm^2 norm_s[0 .. rows), ascending, in units scaled by s; a
// stored row is within min(err, 2^-8 |x|) of its scaled row x = s theta_v,
// bfloat16 rounding each coordinate within 2^-8 relative).  A row whose
// exact distance to the query is at most d_k = sqrt(tau_d) has |x| within
// s d_k of s |theta_q|, so its stored norm lies in that interval widened by
// the rounding bound at its ends, and here also by 2^-15 (s|theta_q| +
// s d_k) for the FP32 rows, 2^-15 relative on the squared norms (FP32 sums)
// and 10^-9 on d_k (the FP64 distances).  Output: the band's rows [a, b).
__global__ void __launch_bounds__(kBlock)
k_knn_band(const float* __restrict__ qtheta, int32_t D, const int32_t* __restrict__ queries,
           const int32_t* __restrict__ rows, int64_t nr, const double* __restrict__ tau_d,
           const float* __restrict__ norm_s, int64_t nrows, double scale, double err,
           int64_t* __restrict__ band) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nr) return;
  const float* tq = qtheta + (int64_t)queries[rows[i]] * D;
  double nq2 = 0.0;
  for (int d = 0; d < D; ++d) nq2 = fma((double)tq[d], (double)tq[d], nq2);
  const double rq = scale * sqrt(nq2), dk = scale * sqrt(tau_d[i]) * (1.0 + 1e-9);
  // a stored (bfloat16) row is within min(err, 2^-8 |x|) of its row x, and
  // x - min(err, 2^-8 x), x + min(err, 2^-8 x) both increase with x
  const double x0 = rq - dk > 0.0 ? rq - dk : 0.0, x1 = rq + dk;
  const double slack = (rq + dk) * 3.0517578125e-05;  // FP32 rows and norms
  const double lo = x0 - fmin(err, x0 * 0.00390625) - slack;
  const double hi = x1 + fmin(err, x1 * 0.00390625) + slack;
  const float lo2 = lo > 0.0 ? (float)(lo * lo * (1.0 - 3.0517578125e-05)) : -1.f;
  const float hi2 = (float)(hi * hi * (1.0 + 3.0517578125e-05));
  // first row with norm >= lo2, first row with norm > hi2
  int64_t a = 0, b = nrows;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (norm_s[m] < lo2) a = m + 1;
    else b = m;
  }
  int64_t e = a, f = nrows;
  while (e < f) {
    const int64_t m = (e + f) >> 1;
    if (norm_s[m] <= hi2) e = m + 1;
    else f = m;
  }
  band[2 * i] = a;
  band[2 * i + 1] = e;
}

// The band form of k_knn_range: work-group (i, g) compares listed query i
// with rows a_i + g*256 + t, stepping by G*256, of its band (vertex sid[p]).
__global__ void __launch_bounds__(kBlock)
k_knn_range_band(const float* __restrict__ theta, int32_t D, const float* __restrict__ qtheta,
                 int32_t exclude_self, const int32_t* __restrict__ queries,
                 const int32_t* __restrict__ rows, const double* __restrict__ tau_d,
                 const int32_t* __restrict__ tau_v, const int64_t* __restrict__ band,
                 const int32_t* __restrict__ sid, uint32_t cap, double* __restrict__ cand_d,
                 int32_t* __restrict__ cand_v, unsigned int* __restrict__ cand_n) {
  extern __shared__ __align__(16) char lds[];
  double* qv = reinterpret_cast<double*>(lds);  // [D]
  const int64_t i = blockIdx.x;
  const int32_t me = queries[rows[i]];
  for (int d = threadIdx.x; d < D; d += kBlock) qv[d] = (double)qtheta[(int64_t)me * D + d];
  __syncthreads();
  const double td = tau_d[i];
  const int32_t tv = tau_v[i];
  const int64_t b = band[2 * i + 1];
  const int64_t stride = (int64_t)gridDim.y * kBlock;
  for (int64_t p = band[2 * i] + (int64_t)blockIdx.y * kBlock + threadIdx.x; p < b; p += stride) {
    const int32_t v = sid[p];
    const float* row = theta + (int64_t)v * D;
    double acc = 0.0;
    for (int d = 0; d < D; ++d) {
      const double delta = qv[d] - (double)row[d];
      acc = fma(delta, delta, acc);
    }
    if ((!exclude_self || v != me) && (acc < td || (acc == td && v <= tv))) {
      const unsigned pos = atomicAdd(&cand_n[i], 1u);
      if (pos < cap) {
        cand_d[i * cap + pos] = acc;
        cand_v[i * cap + pos] = v;
      }
    }
  }
}

// One work-group per listed query: sort its candidates by (d2, id) and
// write the first k to output row rows[i].  A list that overflowed is left
// alone and its index is appended to ov_list.
__global__ void __launch_bounds__(kBlock)
k_knn_cand_select(const int32_t* __restrict__ rows, const double* __restrict__ cand_d,
                  const int32_t* __restrict__ cand_v, const unsigned int* __restrict__ cand_n,
                  uint32_t cap, int32_t k, int32_t* __restrict__ out_ids,
                  double* __restrict__ out_dist, int32_t* __restrict__ ov_list,
                  unsigned long long* __restrict__ ov_n) {
  __shared__ double sd[kSelCap];
  __shared__ int32_t sv[kSelCap];
  const int64_t i = blockIdx.x;
  const unsigned c = cand_n[i];
  const int64_t qi = rows[i];
  if (c > cap) {
    if (threadIdx.x == 0) ov_list[atomicAdd(ov_n, 1ull)] = (int32_t)qi;
    return;
  }
  int P = 2;
  while (P < (int)c) P <<= 1;
  for (int j = threadIdx.x; j < P; j += kBlock) {
    const bool ok = j < (int)c;
    sd[j] = ok ? cand_d[i * cap + j] : INFINITY;
    sv[j] = ok ? cand_v[i * cap + j] : 0x7FFFFFFF;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = threadIdx.x; j < (P >> 1); j += kBlock) {
        const int lo = ((j & ~(stride - 1)) << 1) | (j & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const double a = sd[lo], b = sd[hi];
        const int32_t x = sv[lo], y = sv[hi];
        if (pair_less(b, y, a, x) == asc) {
          sd[lo] = b;
          sd[hi] = a;
          sv[lo] = y;
          sv[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < k; j += kBlock) {
    const bool ok = j < (int)c;
    out_ids[qi * k + j] = ok ? sv[j] : -1;
    out_dist[qi * k + j] = ok ? sqrt(sd[j]) : INFINITY;
  }
}

}  // namespace

int launch_knn_fp64(const float* theta, int32_t n, int32_t D, const float* qtheta,
                    bool exclude_self, const int32_t* queries, const int32_t* rows, int64_t nq,
                    int32_t k, int32_t* out_ids, double* out_dist, hipStream_t s);

size_t knn_range_bytes(int64_t nr) {
  return (sizeof(double) + sizeof(int32_t)) * (size_t)nr * kSelCap + sizeof(unsigned) * nr +
         sizeof(int32_t) * nr + 2 * sizeof(int64_t) * nr + 256;
}

// Exact recompute of listed queries from a known bound: rows[i] (i < nr)
// names the output row of query queries[rows[i]], and (tau_d[i], tau_v[i])
// is an exact (d2, id) pair that at least k rows reach.  work: device
// memory of knn_range_bytes(nr) bytes; nb: the norm-ordered copy whose
// band of each query is scanned.  A list keeps up to min(cap, 4096)
// candidates; lists that outgrow it are recomputed by the full brute force
// (one host synchronisation).
int launch_knn_recompute(const float* theta, int32_t n, int32_t D, const float* qtheta,
                         bool exclude_self, const int32_t* queries, const int32_t* rows,
                         int64_t nr, const double* tau_d, const int32_t* tau_v, int32_t k,
                         int num_cus, void* work, unsigned long long* ov_n_dev,
                         int32_t* out_ids, double* out_dist, hipStream_t s, uint32_t cap,
                         const KnnBand* nb) {
  cap = std::min<uint32_t>(cap, kSelCap);
  if (nr <= 0) return 0;
  if (!nb) return (int)hipErrorInvalidValue;
  char* w = static_cast<char*>(work);
  double* cand_d = reinterpret_cast<double*>(w);
  int32_t* cand_v = reinterpret_cast<int32_t*>(cand_d + (size_t)nr * kSelCap);
  int64_t* band = reinterpret_cast<int64_t*>(cand_v + (size_t)nr * kSelCap);  // 8-aligned
  unsigned* cand_n = reinterpret_cast<unsigned*>(band + 2 * nr);
  int32_t* ov_list = reinterpret_cast<int32_t*>(cand_n + nr);
  hipError_t e = hipMemsetAsync(cand_n, 0, sizeof(unsigned) * nr, s);
  if (e != hipSuccess) return (int)e;
  e = hipMemsetAsync(ov_n_dev, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return (int)e;
  {
    // rows in the norm order of a sorted copy, each query within its band
    k_knn_band<<<(unsigned)((nr + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        qtheta, D, queries, rows, nr, tau_d, nb->norm_s, nb->rows, nb->scale, nb->err, band);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    // at least 64 work-groups per query (up to 256 for a few queries):
    // bands differ by orders of magnitude (a hub's spans most rows), and
    // the work-groups of a narrow band find nothing to do and end at once
    const int64_t gy = std::max<int64_t>(
        64, std::min<int64_t>(256, (4 * (int64_t)num_cus + nr - 1) / nr));
    const size_t lds = sizeof(double) * D;
    k_knn_range_band<<<dim3((unsigned)nr, (unsigned)gy), kBlock, lds, s>>>(
        theta, D, qtheta, exclude_self ? 1 : 0, queries, rows, tau_d, tau_v, band, nb->sid, cap,
        cand_d, cand_v, cand_n);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
  }
  k_knn_cand_select<<<(unsigned)nr, kBlock, 0, s>>>(rows, cand_d, cand_v, cand_n, cap, k,
                                                   out_ids, out_dist, ov_list, ov_n_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  unsigned long long ov = 0;
  e = hipMemcpyAsync(&ov, ov_n_dev, sizeof ov, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return (int)e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return (int)e;
  if (ov == 0) return 0;
  return launch_knn_fp64(theta, n, D, qtheta, exclude_self, queries, ov_list, (int64_t)ov, k,
                         out_ids, out_dist, s);
}

size_t knn_fp64_lds(int D) {
  constexpr int QT = 16;
  return sizeof(double) * QT * D + (sizeof(double) + sizeof(int32_t)) * QT * kBuf +
         sizeof(uint32_t) * (QT + 1) + (sizeof(double) + 2 * sizeof(int32_t)) * QT + 64;
}

// qtheta: the queries' feature rows (theta itself for one graph, the other
// graph's for the cross-graph form, which excludes no row).  rows (may be
// null): the call answers queries[rows[i]] into output row rows[i] for
// i < nq, instead of queries[i] into row i.
int launch_knn_fp64(const float* theta, int32_t n, int32_t D, const float* qtheta,
                    bool exclude_self, const int32_t* queries, const int32_t* rows, int64_t nq,
                    int32_t k, int32_t* out_ids, double* out_dist, hipStream_t s) {
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
                                              rows, nq, k, kp, out_ids, out_dist);
  return (int)hipGetLastError();
}

}  // namespace panther
