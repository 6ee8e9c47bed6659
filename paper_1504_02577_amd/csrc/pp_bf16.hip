// Panther++ nearest neighbours, precision form: a BF16 matrix-core pass
// keeps a candidate pool per query, then an exact FP64 rerank of the pool.
//
// 1. Feature rows are scaled by R (so theta * R is the integer count c) and
//    rounded to bfloat16, zero-padded to 64 columns; counts up to 256 are
//    exact in bfloat16, and their products and sums stay exact in the FP32
//    accumulator.  FP32 row norms come from the same bfloat16 values.  The
//    rows are stored in ascending order of norm (with each row's original
//    id), and every call orders its queries by norm too.
// 2. Pool pass: a work-group owns 16 or 32 queries of neighbouring norms and
//    scans chunks of 64 database rows outward from the chunk where their
//    median norm falls, alternately upward and downward.  Each wavefront
//    computes its queries' dot products with 16 rows per chunk with
//    v_mfma_f32_16x16x32_bf16 (query operands stay in registers), turns
//    them into d2~ = |b_q|^2 + |b_v|^2 - 2 <b_q, b_v>, and appends (d2~, v)
//    keys below the query's threshold to that query's pool buffer in global
//    memory.  Buffers that could overflow are cut back to the pool size P,
//    which sets the threshold to the P-th best key.  Keys are (float bits
//    of d2~, original id), so ties break by id exactly as in the exact
//    order.  The reverse triangle inequality bounds d2~ below by the gap
//    between the two norms (less the rounding bound below): once a
//    direction reaches rows whose norms lie outside every query's band
//    (norm +- threshold radius), it stops -- those rows could not enter
//    any pool.  The pool is thus the P smallest keys over all rows, the
//    same set a full scan gives, from a fraction of the rows.
// 3. Rerank: one work-group per query recomputes the exact FP64 squared
//    distance (one fma per coordinate, coordinate order) of every pool
//    member (one member per thread), sorts by (d2, id) and writes the
//    first k.  It also records how
//    many of the final ids the pool order already had in its first k, and
//    the relative error of d2~ / R^2 against d2 on the returned neighbours.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>


#include "../../include/panther.h"
#include "common.h"
#include "runtime.h"

using namespace panther;

namespace {

constexpr int kBlock = 256;
constexpr int kDP = 64;        // padded feature width in bfloat16
constexpr int kChunk = 64;     // database rows per chunk (16 per wavefront)
constexpr int kTrip = 4;        // chunks per loop trip (register ring of operands)
constexpr int kCheckEvery = 16;  // chunks between pool compaction checks (whole trips)
constexpr int kBoundChunks = 32;  // chunks of the bound pass before a sliced scan

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// FP32 norm of the scaled bfloat16 row of each vertex, as sort keys (the
// bits of a non-negative float order like the float), with the vertex ids
__global__ void __launch_bounds__(kBlock)
k_bf16_norm_keys(const float* __restrict__ theta, int32_t n, int32_t D, float s,
                 uint32_t* __restrict__ keys, int32_t* __restrict__ ids) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  float acc = 0.f;
  for (int d = 0; d < D; ++d) {
    const float f = (float)(__bf16)(theta[(int64_t)v * D + d] * s);
    acc = fmaf(f, f, acc);
  }
  keys[v] = __float_as_uint(acc);
  ids[v] = v;
}

// Rows of norm 0 are all equal, and a zero row is at d2~ = |b_q|^2 from
// every query, so only the zero rows of the smallest ids can enter a pool:
// beyond the first kZeroKeep of them (P <= 1024, plus the query itself),
// every zero row has at least P zero rows of smaller id, hence of smaller
// key, and the pool of the rows kept equals the pool of all rows.
constexpr int64_t kZeroKeep = 1025;

__global__ void __launch_bounds__(kBlock)
k_count_zero(const uint32_t* __restrict__ keys, int64_t n, unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool z = i < n && keys[i] == 0u;
  const uint64_t m = __ballot(z);
  if ((threadIdx.x & (kWave - 1)) == 0 && m) atomicAdd(out, (unsigned long long)__popcll(m));
}

// bf16 rows (scaled by s) in ascending norm order.  Source position i of
// the sorted order (vertex order[i]) goes to row i, or i - drop past the
// kept zero rows [0, zk); the dropped zero rows [zk, zk + drop) keep rank 0
// (a zero row, the same operand).  sid[row] is the row's vertex, rank[v]
// its row.
__global__ void __launch_bounds__(kBlock)
k_bf16_rows_sorted(const float* __restrict__ theta, int32_t n, int32_t D, float s,
                   const int32_t* __restrict__ order, int64_t zk, int64_t drop,
                   int32_t* __restrict__ sid, __bf16* __restrict__ out, float* __restrict__ norm,
                   int32_t* __restrict__ rank) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t v = order[i];
  if (i >= zk && i < zk + drop) {
    rank[v] = 0;
    return;
  }
  const int64_t row = i < zk ? i : i - drop;
  float acc = 0.f;
  for (int d = 0; d < kDP; ++d) {
    const __bf16 b = d < D ? (__bf16)(theta[(int64_t)v * D + d] * s) : (__bf16)0.f;
    out[row * kDP + d] = b;
    const float f = (float)b;
    acc = fmaf(f, f, acc);
  }
  norm[row] = acc;
  sid[row] = v;
  rank[v] = (int32_t)row;
}

// padding rows [n_rows, npad): zero, NaN norm, id INT32_MAX
__global__ void __launch_bounds__(kBlock)
k_bf16_pad_rows(int64_t n_rows, int64_t npad, int32_t* __restrict__ sid, __bf16* __restrict__ out,
                float* __restrict__ norm) {
  const int64_t i = n_rows + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= npad) return;
  for (int d = 0; d < kDP; ++d) out[i * kDP + d] = (__bf16)0.f;
  norm[i] = __builtin_nanf("");
  sid[i] = 0x7FFFFFFF;
}

// sort keys for the queries: norm of each query position's operand
__global__ void __launch_bounds__(kBlock)
k_query_norm_keys(const float* __restrict__ norm, const int32_t* __restrict__ rank,
                  const float* __restrict__ qnorm, const int32_t* __restrict__ queries, int64_t nq,
                  uint32_t* __restrict__ keys, int32_t* __restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nq) return;
  keys[i] = __float_as_uint(qnorm ? qnorm[i] : norm[rank[queries[i]]]);
  pos[i] = (int32_t)i;
}

// bf16 rows of the queries' own features (another graph's theta), scaled
// by the database's s, gathered by query position
__global__ void __launch_bounds__(kBlock)
k_bf16_query_rows(const float* __restrict__ theta_q, int32_t D, const int32_t* __restrict__ queries,
                  int64_t nq, float s, __bf16* __restrict__ out, float* __restrict__ norm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nq) return;
  const int32_t q = queries[i];
  float acc = 0.f;
  for (int d = 0; d < kDP; ++d) {
    const __bf16 b = d < D ? (__bf16)(theta_q[(int64_t)q * D + d] * s) : (__bf16)0.f;
    out[i * kDP + d] = b;
    const float f = (float)b;
    acc = fmaf(f, f, acc);
  }
  norm[i] = acc;
}

// Database bounds for the pool certificate, each rounded up to float and
// combined by an integer max of the (non-negative) float bits:
// out[0] >= max_v |theta_v|, out[1] >= max_v |bf16(theta_v * s) - theta_v * s|
// (the rounding error of a scaled row, in scaled units).
__global__ void __launch_bounds__(kBlock)
k_row_bounds(const float* __restrict__ theta, int32_t n, int32_t D, float s, unsigned int* out) {
  const int32_t v = blockIdx.x * kBlock + threadIdx.x;
  float f = 0.f, g = 0.f;
  if (v < n) {
    double a = 0.0, b = 0.0;
    for (int d = 0; d < D; ++d) {
      const float t = theta[(int64_t)v * D + d];
      const double x = (double)t;
      a = fma(x, x, a);
      const double y = (double)(t * s);
      const double r = (double)(float)(__bf16)(t * s) - y;
      b = fma(r, r, b);
    }
    f = (float)(sqrt(a) * (1.0 + 1.0 / (1 << 20)));
    g = (float)(sqrt(b) * (1.0 + 1.0 / (1 << 20)));
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const float o = __shfl_xor(f, off, kWave);
    f = o > f ? o : f;
    const float p = __shfl_xor(g, off, kWave);
    g = p > g ? p : g;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(out, __float_as_uint(f));
    atomicMax(out + 1, __float_as_uint(g));
  }
}

__global__ void k_fill_u64(unsigned long long* a, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

// ascending bitonic sort of cnt keys (padded with ~0) by one wavefront
__device__ void wave_sort_keys(uint64_t* a, int cnt) {
  const int lane = threadIdx.x & (kWave - 1);
  int P = 2;
  while (P < cnt) P <<= 1;
  for (int i = cnt + lane; i < P; i += kWave) a[i] = ~0ull;
  wsync();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (P >> 1); i += kWave) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t x = a[lo], y = a[hi];
        if ((x > y) == asc) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      wsync();
    }
  }
}

// The P smallest of the c > P distinct keys a[0..c) by one wavefront: an
// MSD radix select (8-bit digits, histogram in `hist`, 256 words) finds the
// P-th smallest key T, then a[0..P) is compacted in place to the keys <= T
// (in input order).  Returns T.
__device__ uint64_t wave_select_cut(uint64_t* a, int c, int P, uint32_t* hist) {
  const int lane = threadIdx.x & (kWave - 1);
  uint64_t prefix = 0;  // digits fixed so far
  int need = P;         // rank of T within the current class (1-based)
  for (int shift = 56; shift >= 0; shift -= 8) {
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[lane * 4 + b] = 0u;
    wsync();
    const uint64_t hi_mask = shift == 56 ? 0ull : (~0ull << (shift + 8));
    for (int i = lane; i < c; i += kWave) {
      const uint64_t x = a[i];
      if ((x & hi_mask) == prefix) atomicAdd(&hist[(uint32_t)(x >> shift) & 255u], 1u);
    }
    wsync();
    // lane l owns digits 4l .. 4l+3; the digit where the running count
    // reaches `need` holds T
    uint32_t h[4], sum = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      h[b] = hist[lane * 4 + b];
      sum += h[b];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
    uint32_t below = inc - sum;
    int dsel = -1;
    uint32_t below_sel = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (dsel < 0 && below < (uint32_t)need && below + h[b] >= (uint32_t)need) {
        dsel = lane * 4 + b;
        below_sel = below;
      }
      below += h[b];
    }
    const uint64_t m = __ballot(dsel >= 0);
    const int src = __ffsll((long long)m) - 1;
    const int d = __shfl(dsel, src, kWave);
    need -= (int)__shfl(below_sel, src, kWave);
    prefix |= (uint64_t)d << shift;
    wsync();
  }
  const uint64_t T = prefix;
  // in-place compaction: a position is written only after it was read
  int base = 0;
  for (int i0 = 0; i0 < c; i0 += kWave) {
    const int i = i0 + lane;
    const uint64_t x = i < c ? a[i] : ~0ull;
    const bool keep = i < c && x <= T;
    const uint64_t bm = __ballot(keep);
    if (keep) a[base + __popcll(bm & ((1ull << lane) - 1ull))] = x;
    base += __popcll(bm);
    wsync();
  }
  return T;
}

struct PoolArgs {
  const __bf16* rows;    // [npad][64] database rows in ascending norm order
  const float* norm;     // [npad] their FP32 norms (NaN past n)
  const int32_t* sid;    // [npad] original id of each row (INT32_MAX past n)
  const int32_t* rank;   // [vertices] row of each original id (a zero row if dropped)
  int32_t n;             // database rows (zero rows past the kept ones dropped)
  int64_t nchunks;       // chunks of rows (whole trips); chunk nchunks is all padding
  const int32_t* queries;
  const int32_t* q_order;// query positions in ascending order of operand norm
  int64_t nq;
  int32_t P;             // pool size (power of two, <= 1024)
  int32_t cap;           // buffer entries per (query, slice): 2P + kCheckEvery * kChunk
  int32_t slices;        // work-groups per query tile (grid.y), interleaved over chunks
  int32_t sort_cap;      // per-wave buffer entries (>= cap, and >= the sort's P)
  uint64_t* buf;         // [nq][slices][cap] pool buffers, by sorted index
  uint64_t* part;        // [nq][slices][P] slice pools (slices > 1), by sorted index
  int32_t* pool_ids;     // [nq][P] result by query position, ascending key order, -1 padded
  float* pool_d2;        // [nq][P]
  // query operands: the database's own rows (row rank[q]), or (cross
  // form) qrows[i] / qnorm[i] gathered per query position i
  const __bf16* qrows;
  const float* qnorm;
  int32_t q_by_pos;
  int32_t exclude_self;  // single graph: the query's own row is no candidate
  // slices > 1: per query (sorted index), the smallest P-th best key any
  // slice has reached so far -- an upper bound on the query's P-th best key
  // overall, so every slice may drop keys at or above it
  unsigned long long* gtau;
  unsigned long long* stat_products;  // += (query, row) products computed
  // bound pass: stop after max_chunks chunks and publish, for each full
  // pool, the key after its P-th to gtau instead of writing pools (at
  // least P rows have keys below it: a valid exclusive bound)
  int32_t max_chunks;    // 0: no limit
  int32_t bound_only;
};

// Norm band of one query for the current float threshold t (squared
// units).  A row whose exact norm x has |x - |b_q|| = g satisfies
// d2~ >= g^2 - delta with delta <= 2^-15 (|b_q|^2 + x^2) (the rounding
// bound of d2~), so d2~ > t, and the row cannot enter the pool, once
// g^2 > (t + 2^-13 |b_q|^2)(1 + 2^-13).  With rho^2 = (t + 2^-12 qn)(1 +
// 2^-12) that holds for computed norms (FP32 sums of 64 squares, relative
// error below 2^-17 after the square root) outside
//   [ (sqrt(qn)(1 - 2^-16) - rho)^2, (sqrt(qn)(1 + 2^-16) + rho)^2 ],
// widened once more by 2^-12 relative.  lo2 = 0 when the band reaches 0.
__device__ __forceinline__ void norm_band(float qn, float t, float& lo2, float& hi2) {
  if (!(t < INFINITY)) {
    lo2 = 0.f;
    hi2 = INFINITY;
    return;
  }
  const float rq = sqrtf(qn);
  const float rho = sqrtf((t + qn * 2.44140625e-4f) * (1.f + 2.44140625e-4f));
  const float hi = rq * (1.f + 1.52587890625e-5f) + rho;
  const float lo = rq * (1.f - 1.52587890625e-5f) - rho;
  hi2 = hi * hi * (1.f + 2.44140625e-4f);
  lo2 = lo > 0.f ? lo * lo * (1.f - 2.44140625e-4f) : 0.f;
}

// grid (query tiles of QW, slices)
template <int QW>
__global__ void __launch_bounds__(kBlock)
k_pp_pool(PoolArgs A) {
  constexpr int kTiles = QW / 16;  // 16-query MFMA tiles per wavefront
  __shared__ uint32_t cnt[QW];
  __shared__ uint64_t tau[QW];
  __shared__ float tauf_s[QW];  // float part of tau, for the prefilter
  __shared__ int32_t qid[QW];
  __shared__ int32_t qpos[QW];
  __shared__ float qn_s[QW];
  __shared__ uint32_t s_band[2];  // float bits: band of the whole tile [lo2, hi2]
  __shared__ int32_t s_dir[2];    // directions still open: up, down
  __shared__ int64_t s_c0;        // chunk of the tile's median norm
  extern __shared__ __align__(16) uint64_t sortmem[];  // [waves][cap]
  __shared__ uint32_t s_hist[kBlock / kWave][256];     // per-wave radix select
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t q0 = (int64_t)blockIdx.x * QW;  // sorted index of the tile's first query
  const int slice = blockIdx.y;
  const int S = A.slices;
  const int P = A.P, cap = A.cap;
  const int check_every = kCheckEvery;
  const int nvalid = (int)(A.nq - q0 < QW ? A.nq - q0 : QW);
  for (int i = threadIdx.x; i < QW; i += kBlock) {
    const int32_t pos = i < nvalid ? A.q_order[q0 + i] : -1;
    const int32_t q = pos >= 0 ? A.queries[pos] : -1;
    qid[i] = q;
    qpos[i] = pos;
    qn_s[i] = q >= 0 ? (A.q_by_pos ? A.qnorm[pos] : A.norm[A.rank[q]]) : 0.f;
    cnt[i] = 0u;
    // start from the shared bound when there is one (a bound pass or
    // other slices may have set it)
    const unsigned long long gb =
        q >= 0 && A.gtau && !A.bound_only
            ? __hip_atomic_load(&A.gtau[q0 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
            : ~0ull;
    tau[i] = gb;
    tauf_s[i] = q < 0 ? -1.f  // a missing query matches nothing
                      : (gb == ~0ull ? INFINITY : __uint_as_float((uint32_t)(gb >> 32)));
  }
  if (threadIdx.x == 0) {
    s_band[0] = 0u;
    s_band[1] = __float_as_uint(INFINITY);
    s_dir[0] = s_dir[1] = 1;
  }
  __syncthreads();
  // start chunk: where the median query norm falls among the sorted rows
  // (a 256-way search for the first row with norm >= target: rows below
  // lo are below it, and row hi is n or not below it)
  {
    const float target = qn_s[(nvalid - 1) / 2];
    int64_t lo = 0, hi = A.n;
    while (lo < hi) {
      const int64_t step = (hi - lo + kBlock - 1) / kBlock;
      const int64_t idx = lo + (int64_t)threadIdx.x * step;
      const int below = idx < hi && A.norm[idx] < target;
      const int nb = __syncthreads_count(below);  // the probes below form a prefix
      if (nb == 0) {
        hi = lo;
      } else {
        const int64_t last = lo + (int64_t)(nb - 1) * step;  // last probe below
        lo = last + 1;
        hi = last + step < hi ? last + step : hi;
      }
    }
    if (threadIdx.x == 0) {
      int64_t c = lo / kChunk;
      if (c >= A.nchunks) c = A.nchunks - 1;
      s_c0 = c;
    }
    __syncthreads();
  }
  const int64_t c0 = __builtin_amdgcn_readfirstlane((int)s_c0);
  // query operands: tile m, k-step ks -> 8 bf16 of row (m*16 + l%16)
  bf16x8 a[kTiles][2];
#pragma unroll
  for (int m = 0; m < kTiles; ++m) {
    const int32_t q = qid[m * 16 + (lane & 15)];
    const __bf16* qr = A.q_by_pos ? A.qrows + (int64_t)qpos[m * 16 + (lane & 15)] * kDP
                                  : A.rows + (int64_t)(q >= 0 ? A.rank[q] : 0) * kDP;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      if (q >= 0) {
        a[m][ks] = *reinterpret_cast<const bf16x8*>(qr + ks * 32 + 8 * (lane >> 4));
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[m][ks][j] = (__bf16)0.f;
      }
    }
  }
  // database rows: 16 per wavefront and chunk, row (l%16) as the MFMA's A
  // operand, so that lane l receives the products of query m*16 + l%16
  // with rows 4*(l/16) .. 4*(l/16)+3 of its wavefront's 16.  The row arrays
  // are padded to whole trips of chunks plus one chunk (zero rows, NaN
  // norms), so every load is unconditional; a padding row's d2~ is NaN and
  // passes no test, and chunk -1 (none) is the all-padding chunk.
  auto load_b = [&](int64_t c, bf16x8 (&bb)[2], floatx4& nvv, int4& idv) {
    const int64_t cb = (c >= 0 ? c : A.nchunks) * kChunk;  // -1: the all-padding chunk
    const int64_t v = cb + wid * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      bb[ks] = *reinterpret_cast<const bf16x8*>(A.rows + v * kDP + ks * 32 + 8 * (lane >> 4));
    nvv = *reinterpret_cast<const floatx4*>(A.norm + cb + wid * 16 + 4 * (lane >> 4));
    idv = *reinterpret_cast<const int4*>(A.sid + cb + wid * 16 + 4 * (lane >> 4));
  };
  // Per lane and tile: the norm qn and float threshold t of its query, and
  // the prefilter bound tm on u = nv - 2 <b_q, b_v> (one rounding, by fma):
  // d2~ = fl(u + qn) <= t implies u <= fl(t - qn) + 2^-21 (|t| + qn), so
  // the prefilter drops no row that the exact test would keep.  Kept in
  // registers; refreshed after every check.
  float qnr[kTiles], tfr[kTiles], tmr[kTiles];
  auto refresh = [&]() {
#pragma unroll
    for (int m = 0; m < kTiles; ++m) {
      tfr[m] = tauf_s[m * 16 + (lane & 15)];
      tmr[m] = (tfr[m] - qnr[m]) + (fabsf(tfr[m]) + qnr[m]) * 4.76837158203125e-7f;
    }
  };
  int32_t qidr[kTiles];  // -1: no query (its threshold -1 passes nothing)
#pragma unroll
  for (int m = 0; m < kTiles; ++m) {
    qnr[m] = qn_s[m * 16 + (lane & 15)];
    qidr[m] = qid[m * 16 + (lane & 15)];
  }
  refresh();
  // one chunk: products, prefilter, appends
  auto chunk = [&](const bf16x8 (&bc)[2], const floatx4& nvc, const int4& idc) {
    floatx4 acc[kTiles];
#pragma unroll
    for (int m = 0; m < kTiles; ++m) {
      acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bc[0], a[m][0], acc[m], 0, 0, 0);
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bc[1], a[m][1], acc[m], 0, 0, 0);
    }
    // per tile: does any lane's smallest u pass the prefilter?
    uint64_t tile_hit[kTiles], any_hit = 0ull;
#pragma unroll
    for (int m = 0; m < kTiles; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][r] = __builtin_fmaf(-2.f, acc[m][r], nvc[r]);  // u
      const float mn = fminf(fminf(acc[m][0], acc[m][1]), fminf(acc[m][2], acc[m][3]));
      tile_hit[m] = __ballot(mn <= tmr[m]);
      any_hit |= tile_hit[m];
    }
    if (any_hit != 0ull) {
      const int32_t ids[4] = {idc.x, idc.y, idc.z, idc.w};
#pragma unroll
      for (int m = 0; m < kTiles; ++m) {
        if (tile_hit[m] == 0ull) continue;
        const int ql = m * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int32_t v = ids[r];
          // d2~ = fl(u + qn); a negative rounding result counts as 0 (the
          // test d2 <= t with t >= 0 is the same before and after the clamp)
          const float raw = acc[m][r] + qnr[m];
          if (raw <= tfr[m] && (!A.exclude_self || qidr[m] != v)) {
            const float d2 = raw > 0.f ? raw : 0.f;
            const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)v;
            // below the threshold's float part the key is below the
            // threshold; at equality the ids decide
            if (d2 < tfr[m] || key < tau[ql]) {
              const uint32_t pos = atomicAdd(&cnt[ql], 1u);
              A.buf[((q0 + ql) * S + slice) * cap + pos] = key;
            }
          }
        }
      }
    }
  };
  // Chunk sequence of this slice: upward c0 + slice, c0 + slice + S, ...
  // and downward c0 - 1 - slice, c0 - 1 - slice - S, ..., alternating while
  // both directions are open; -1 when none is.  Every wavefront runs the
  // same (uniform) sequence.
  int up_on = 1, down_on = 1;
  int64_t nu = 0, nd = 0;
  auto next_chunk = [&]() -> int64_t {
    const int64_t cu = c0 + slice + (int64_t)S * nu;
    const int64_t cd = c0 - 1 - slice - (int64_t)S * nd;
    up_on = up_on && cu < A.nchunks;  // a direction past its end stays closed
    down_on = down_on && cd >= 0;
    if (up_on && (!down_on || nu <= nd)) {
      ++nu;
      return cu;
    }
    if (down_on) {
      ++nd;
      return cd;
    }
    return -1;
  };
  // operands of four chunks in a register ring: each chunk's loads are
  // issued three chunks before its products (a chunk is short next to a
  // load's latency), and the ring rotates by unrolling, without register
  // copies (a copy of a prefetched operand would force a wait)
  bf16x8 b0[2], b1[2], b2[2], b3[2];
  floatx4 nv0, nv1, nv2, nv3;
  int4 id0, id1, id2, id3;
  load_b(next_chunk(), b0, nv0, id0);
  load_b(next_chunk(), b1, nv1, id1);
  load_b(next_chunk(), b2, nv2, id2);
  int chunk_no = 0;
  while (true) {
    load_b(next_chunk(), b3, nv3, id3);
    chunk(b0, nv0, id0);
    const int64_t c_next = next_chunk();  // the oldest chunk left in the ring
    load_b(c_next, b0, nv0, id0);
    chunk(b1, nv1, id1);
    load_b(next_chunk(), b1, nv1, id1);
    chunk(b2, nv2, id2);
    load_b(next_chunk(), b2, nv2, id2);
    chunk(b3, nv3, id3);
    chunk_no += kTrip;
    // once the sequence returns -1 it stays -1: if the oldest chunk left
    // in the ring is none, so are the two after it
    const bool last = c_next < 0 || (A.max_chunks && chunk_no >= A.max_chunks);
    if (chunk_no % check_every != 0 && !last) continue;
    __threadfence_block();
    __syncthreads();
    // adopt the other slices' bound where it is tighter (one load per query)
    if (A.gtau && !A.bound_only) {
      for (int ql = threadIdx.x; ql < QW; ql += kBlock) {
        if (qid[ql] < 0) continue;
        const unsigned long long gb =
            __hip_atomic_load(&A.gtau[q0 + ql], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gb < tau[ql]) {
          tau[ql] = gb;
          tauf_s[ql] = __uint_as_float((uint32_t)(gb >> 32));
        }
      }
      __syncthreads();
    }
    // cut back buffers that the next check_every chunks could overflow, or
    // (first cut) any buffer past P while its threshold is still open
    // (lane j looks at query wid + 4j; the wave then takes them in turn)
    constexpr int kPerWave = QW / (kBlock / kWave);
    const int qj = wid + (kBlock / kWave) * lane;
    const int cj = lane < kPerWave ? (int)cnt[qj] : 0;
    uint64_t todo = __ballot(lane < kPerWave && cj > P &&
                             (cj > cap - check_every * kChunk || tau[qj] == ~0ull));
    while (todo) {
      const int j = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const int ql = wid + (kBlock / kWave) * j;
      const int c = __shfl(cj, j, kWave);
      uint64_t* g = A.buf + ((q0 + ql) * S + slice) * cap;
      uint64_t* sb = sortmem + (size_t)wid * A.sort_cap;
      for (int i = lane; i < c; i += kWave)
        sb[i] = __hip_atomic_load(&g[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      wsync();
      const uint64_t T = wave_select_cut(sb, c, P, s_hist[wid]);
      for (int i = lane; i < P; i += kWave) g[i] = sb[i];
      if (lane == 0) {
        cnt[ql] = (uint32_t)P;
        if (T < tau[ql]) {
          tau[ql] = T;
          tauf_s[ql] = __uint_as_float((uint32_t)(T >> 32));
        }
        // (a slice keeps its P keys <= tau, so the others may drop keys >=
        // tau; the bound pass keeps nothing and publishes only at its end)
        if (A.gtau && !A.bound_only && qid[ql] >= 0)
          atomicMin(&A.gtau[q0 + ql], (unsigned long long)tau[ql]);
      }
      wsync();
    }
    __threadfence_block();
    __syncthreads();
    // the tile's band: union of its queries' bands (bits of non-negative
    // floats order like the floats)
    if (threadIdx.x == 0) {
      s_band[0] = __float_as_uint(INFINITY);
      s_band[1] = 0u;
    }
    __syncthreads();
    if ((int)threadIdx.x < nvalid) {
      float lo2, hi2;
      norm_band(qn_s[threadIdx.x], tauf_s[threadIdx.x], lo2, hi2);
      atomicMin(&s_band[0], __float_as_uint(lo2));
      atomicMax(&s_band[1], __float_as_uint(hi2));
    }
    __syncthreads();
    // close a direction whose next chunk lies wholly outside the band
    // (norms rise upward: past that chunk every row is outside too)
    if (threadIdx.x == 0) {
      const float lo2 = __uint_as_float(s_band[0]), hi2 = __uint_as_float(s_band[1]);
      int up = up_on, down = down_on;
      const int64_t cu = c0 + slice + (int64_t)S * nu;
      if (up && cu < A.nchunks && A.norm[cu * kChunk] > hi2) up = 0;
      const int64_t cd = c0 - 1 - slice - (int64_t)S * nd;
      if (down && cd >= 0) {
        const int64_t last = cd * kChunk + kChunk - 1 < A.n ? cd * kChunk + kChunk - 1 : A.n - 1;
        if (A.norm[last] < lo2) down = 0;
      }
      s_dir[0] = up;
      s_dir[1] = down;
    }
    __syncthreads();
    up_on = __builtin_amdgcn_readfirstlane(s_dir[0]);
    down_on = __builtin_amdgcn_readfirstlane(s_dir[1]);
    refresh();
    if (last) break;  // the sequence ran dry (both directions closed), or the budget
  }
  if (threadIdx.x == 0)
    atomicAdd(A.stat_products, (unsigned long long)((nu + nd) * kChunk * nvalid));
  if (A.bound_only) {
    for (int ql = wid; ql < QW; ql += kBlock / kWave) {
      const int c = (int)cnt[ql];
      if (qid[ql] < 0 || c < P) continue;
      uint64_t* g = A.buf + ((q0 + ql) * S + slice) * cap;
      uint64_t* sb = sortmem + (size_t)wid * A.sort_cap;
      for (int i = lane; i < c; i += kWave)
        sb[i] = __hip_atomic_load(&g[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      wsync();
      // this pass keeps no pool, so the slices must keep keys equal to T
      // too: publish the next key, T + 1 (ids stay below 2^31)
      const uint64_t T = wave_select_cut(sb, c, P, s_hist[wid]);
      if (lane == 0) atomicMin(&A.gtau[q0 + ql], (unsigned long long)(T + 1ull));
      wsync();
    }
    return;
  }
  // final pools of this slice
  for (int ql = wid; ql < QW; ql += kBlock / kWave) {
    if (qid[ql] < 0) continue;
    const int c = (int)cnt[ql];
    uint64_t* g = A.buf + ((q0 + ql) * S + slice) * cap;
    uint64_t* sb = sortmem + (size_t)wid * A.sort_cap;
    for (int i = lane; i < c; i += kWave)
      sb[i] = __hip_atomic_load(&g[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wsync();
    // one slice: the pool in ascending key order; several: the slice's P
    // best in any order (the merge selects across slices).  The P best are
    // cut first, so the sort needs P (a power of two) entries of buffer.
    if (c > P) (void)wave_select_cut(sb, c, P, s_hist[wid]);
    if (S == 1) wave_sort_keys(sb, c < P ? c : P);
    const int m = c < P ? c : P;
    if (S == 1) {
      const int64_t pos = qpos[ql];
      for (int i = lane; i < P; i += kWave) {
        const bool ok = i < m;
        A.pool_ids[pos * P + i] = ok ? (int32_t)(uint32_t)sb[i] : -1;
        A.pool_d2[pos * P + i] = ok ? __uint_as_float((uint32_t)(sb[i] >> 32)) : INFINITY;
      }
    } else {
      // fixed-length slice pools (unordered), padded with the largest key
      uint64_t* o = A.part + ((q0 + ql) * S + slice) * P;
      for (int i = lane; i < P; i += kWave) o[i] = i < m ? sb[i] : ~0ull;
    }
    wsync();
  }
}

// One work-group per query (sorted index): the P smallest keys over all
// slice pools, written to the query's position.
// Slice pools are P keys long, padded with ~0, which complement to 0: a
// selected 0 is padding.
__global__ void __launch_bounds__(kBlock)
k_pp_merge(PoolArgs A) {
  __shared__ SelectSmem sm;
  const int64_t j = blockIdx.x;  // sorted index; the output row is its position
  const int64_t qi = A.q_order[j];
  const int S = A.slices, P = A.P;
  const uint64_t* base = A.part + j * (int64_t)S * P;
  auto key = [&](int i) { return ~base[i]; };  // larger = better
  const int m = block_select_topk<kBlock>(key, S * P, P, sm);
  for (int i = threadIdx.x; i < P; i += kBlock) {
    const bool ok = i < m && sm.out[i] != 0ull;
    const uint64_t k2 = ok ? ~sm.out[i] : 0ull;
    A.pool_ids[qi * P + i] = ok ? (int32_t)(uint32_t)k2 : -1;
    A.pool_d2[qi * P + i] = ok ? __uint_as_float((uint32_t)(k2 >> 32)) : INFINITY;
  }
}

// per query (work-group): d, v, ap of P entries and up to 256 staged ids
__host__ __device__ constexpr size_t rerank_lds(int P) {
  return (sizeof(double) + sizeof(int32_t) + sizeof(float)) * (size_t)P + sizeof(int32_t) * 256;
}

struct RerankArgs {
  const float* theta;    // [n][D] database rows
  const float* db_max;   // [0] >= max_v |theta_v|, [1] >= max_v of a row's bf16 rounding error
  double scale;          // s: the bf16 rows are bf16(theta * s)
  int32_t* fb_list;      // queries whose pool boundary is not certified
  double* fb_tau_d;      // and their k-th exact pair (d2, id)
  int32_t* fb_tau_v;
  unsigned long long* fb_n;
  int32_t force;         // flag every query whose pool is full
  const float* qtheta;   // query rows by query id (theta itself, or the other graph's)
  int32_t D;
  const int32_t* queries;
  int64_t nq;
  int32_t P, k;
  const int32_t* pool_ids;
  const float* pool_d2;
  float inv_s2;          // 1 / s^2: scale of d2~ back to theta units
  int32_t* out_ids;
  double* out_dist;
  unsigned long long* stat_hits;   // sum over queries of pre-rerank hits
  unsigned long long* stat_err;    // max relative error (bits of a double >= 0)
  unsigned long long* stat_ret;    // sum over queries of returned neighbours
};

// one wavefront per query
__global__ void __launch_bounds__(kBlock)
k_pp_rerank(RerankArgs A) {
  // one work-group per query: d[P], v[P], ap[P], first[256]
  extern __shared__ __align__(16) char rr_lds[];
  __shared__ double qv[kDP];
  __shared__ unsigned int s_valid, s_hits;
  __shared__ unsigned long long s_err;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t qi = blockIdx.x;
  const int32_t q = A.queries[qi];
  const int P = A.P, D = A.D;
  const float* tq = A.qtheta + (int64_t)q * D;
  double* d = reinterpret_cast<double*>(rr_lds);
  int32_t* v = reinterpret_cast<int32_t*>(d + P);
  float* ap = reinterpret_cast<float*>(v + P);
  int32_t* first = reinterpret_cast<int32_t*>(ap + P);
  if ((int)threadIdx.x < D) qv[threadIdx.x] = (double)tq[threadIdx.x];
  if (threadIdx.x == 0) {
    s_valid = 0u;
    s_hits = 0u;
    s_err = 0ull;
  }
  __syncthreads();
  // every member's row at once (one member per thread, all loads of a
  // thread's row independent): the exact chain of the oracle
  unsigned my_valid = 0;
  for (int i = threadIdx.x; i < P; i += kBlock) {
    const int32_t c = A.pool_ids[qi * P + i];
    double sacc = INFINITY;
    if (c >= 0) {
      const float* tv = A.theta + (int64_t)c * D;
      sacc = 0.0;
      for (int j = 0; j < D; ++j) {
        const double delta = qv[j] - (double)tv[j];
        sacc = fma(delta, delta, sacc);
      }
      ++my_valid;
    }
    d[i] = sacc;
    v[i] = c >= 0 ? c : 0x7FFFFFFF;
    ap[i] = A.pool_d2[qi * P + i];
  }
  if (my_valid) atomicAdd(&s_valid, my_valid);
  __syncthreads();
  // sort (d, v) ascending; the approximate values ride along
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += kBlock) {
        const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));  // stride: power of two
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const double x = d[lo], y = d[hi];
        const int32_t xv = v[lo], yv = v[hi];
        const bool gt = x > y || (x == y && xv > yv);
        if (gt == asc) {
          d[lo] = y;
          d[hi] = x;
          v[lo] = yv;
          v[hi] = xv;
          const float t = ap[lo];
          ap[lo] = ap[hi];
          ap[hi] = t;
        }
      }
      __syncthreads();
    }
  }
  const int valid = (int)s_valid;
  const int k = A.k;
  const int m = valid < k ? valid : k;
  // the pool order's first m ids (pre-rerank top k: the pool is in key order)
  for (int i = threadIdx.x; i < m; i += kBlock) first[i] = A.pool_ids[qi * P + i];
  __syncthreads();
  unsigned hits = 0;
  double err = 0.0;
  for (int j = threadIdx.x; j < k; j += kBlock) {
    const bool ok = j < m;
    A.out_ids[qi * k + j] = ok ? v[j] : -1;
    A.out_dist[qi * k + j] = ok ? sqrt(d[j]) : INFINITY;
    if (ok) {
      // was this id within the first k of the pool order?
      for (int i = 0; i < m; ++i) hits += (first[i] == v[j]) ? 1u : 0u;
      const double approx = (double)ap[j] * (double)A.inv_s2;
      const double den = d[j] > (double)A.inv_s2 ? d[j] : (double)A.inv_s2;
      const double e = fabs(approx - d[j]) / den;
      err = e > err ? e : err;
    }
  }
  if (hits) atomicAdd(&s_hits, hits);
  if (err > 0.0) atomicMax(&s_err, (unsigned long long)__double_as_longlong(err));  // err >= 0
  __syncthreads();
  if (threadIdx.x >= kWave) return;  // the first wavefront finishes the query
  if (lane == 0) {
    atomicAdd(A.stat_ret, (unsigned long long)m);
    atomicAdd(A.stat_hits, (unsigned long long)s_hits);
    atomicMax(A.stat_err, s_err);
  }
  // Certificate (in units of the scaled rows x = theta * s).  Every vertex
  // outside the pool has a pool key at least the pool's largest, so its
  // computed d2~ >= a_P^2.  A vertex with |x_v| > |x_q| + s d_k is farther
  // than d_k by the triangle inequality; only the others ("near" rows)
  // need a bound.  In general the computed d2~ = |b_q|^2 + |b_v|^2 -
  // 2 <b_q, b_v> over the bfloat16 rows b errs from |b_q - b_v|^2 by at
  // most delta = 2^-15 (|b_q|^2 + |b_v|^2) (about 132 FP32 roundings of
  // those magnitudes, with margin), and |b - x| <= r per row (r_q computed
  // here; r_v <= E for every row, and <= 2^-8 |x_v| <= 2^-8 (|x_q| + s d_k)
  // for a near row).  Rows of counts are integral in bfloat16 (a count
  // below 256 stays itself, a larger one rounds to an even integer), so
  // when b_q is integral too and |b_q|^2 + |b_v|^2 < 2^23 the FP32
  // evaluation is exact (delta = 0: the result |b_q - b_v|^2 and every
  // partial sum stay integers below 2^24).  When moreover |x_q| + s d_k < 255,
  // every near row has coordinates below 255, which bfloat16 keeps exactly
  // (x is count * (1 +- 2^-23)), so r_v <= 2^-22 (|x_q| + s d_k).  If
  // sqrt(a_P^2 - delta) - r_q - r_v > s d_k, no outside vertex can enter
  // the top k, ties included.  In that last case with d_k = 0 the k results
  // are rows equal to the query's, each with d2~ = 0 in the pool in id
  // order, so it is certified too.  Otherwise the query is recomputed
  // exactly: every row within its k-th exact pair (d_k, id) is a candidate.
  double nq2 = 0.0, rq2 = 0.0;
  bool q_int = true;
  const float sf = (float)A.scale;
  for (int j = lane; j < A.D; j += kWave) {
    nq2 = fma((double)tq[j], (double)tq[j], nq2);
    const float b = (float)(__bf16)(tq[j] * sf);
    const double r = (double)b - (double)(tq[j] * sf);
    rq2 = fma(r, r, rq2);
    q_int = q_int && b == floorf(b);
  }
  for (int off = 32; off > 0; off >>= 1) {
    nq2 += __shfl_xor(nq2, off, kWave);
    rq2 += __shfl_xor(rq2, off, kWave);
  }
  q_int = __ballot(!q_int) == 0ull;
  if (lane == 0) {
    const bool full = A.pool_ids[qi * P + P - 1] >= 0;
    bool ok = !full || m < k;
    if (!ok && !A.force) {
      const double s = A.scale, dk = s * sqrt(d[k - 1]);
      const double xq = s * sqrt(nq2), M = s * (double)A.db_max[0], E = (double)A.db_max[1];
      const double reach = xq + dk;
      const bool small = q_int && reach < 255.0;
      if (small && d[k - 1] == 0.0) {
        ok = true;
      } else {
        const double bq = xq * (1.0 + 1.0 / 256.0);
        const double bv = fmin(M, reach) * (1.0 + 1.0 / 256.0);
        // integral rows with |b_q|^2 + |b_v|^2 < 2^23: every partial sum
        // of the evaluation (in any order) is an integer below 2^24, exact
        // in FP32
        const bool exact = q_int && bq * bq + bv * bv < 8388608.0;
        const double delta = exact ? 0.0 : 3.0517578125e-05 * (bq * bq + bv * bv);
        const double rv = small ? 2.384185791015625e-07 * reach : fmin(E, reach / 128.0);
        const double a2 = (double)A.pool_d2[qi * P + P - 1];
        // r was measured against the FP32 product theta * s, which is within
        // 2^-24 of the exact scaled row
        const double lower = sqrt(fmax(a2 - delta, 0.0)) - sqrt(rq2) * (1.0 + 1e-6) - rv -
                             1.2e-7 * (xq + bv);
        ok = lower > dk * (1.0 + 1e-9);
      }
    }
    if (!ok) {
      const unsigned long long at = atomicAdd(A.fb_n, 1ull);
      A.fb_list[at] = (int32_t)qi;
      A.fb_tau_d[at] = d[k - 1];
      A.fb_tau_v[at] = v[k - 1];
    }
  }
}


// Scratch bytes of sort_pairs for n pairs.
size_t sort_pairs_bytes(int64_t n) {
  const uint64_t tiles = radix_tiles_pairs((uint64_t)std::max<int64_t>(n, 1));
  const size_t hist = 256 * (size_t)tiles;
  return sizeof(uint32_t) * hist + sizeof(uint64_t) * (hist + 1) + scan_temp_bytes((int64_t)hist) +
         64 + 2 * sizeof(uint32_t) * (size_t)std::max<int64_t>(n, 1) + 4 * 256;
}

// Ascending, stable sort of n (uint32 key, int32 value) pairs by the same
// LSD radix passes as the index build (four 8-bit digits); tmp holds the
// per-tile histograms, their scan, the pair count and a ping-pong copy.
// kin and vin are only read.
int sort_pairs(panther_ctx* c, DevBuf& tmp, const uint32_t* kin, uint32_t* kout,
               const int32_t* vin, int32_t* vout, int64_t n, hipStream_t s) {
  if (n <= 0) return PANTHER_OK;
  const uint64_t tiles = radix_tiles_pairs((uint64_t)n);
  const size_t hist_n = 256 * (size_t)tiles;
  TRY(ctx_ensure(c, tmp, sort_pairs_bytes(n), "sort scratch"));
  char* p = static_cast<char*>(tmp.p);
  uint32_t* hist = reinterpret_cast<uint32_t*>(p);
  p += sizeof(uint32_t) * hist_n;
  p = reinterpret_cast<char*>(((uintptr_t)p + 255) & ~(uintptr_t)255);
  uint64_t* offs = reinterpret_cast<uint64_t*>(p);
  p += sizeof(uint64_t) * (hist_n + 1);
  p = reinterpret_cast<char*>(((uintptr_t)p + 255) & ~(uintptr_t)255);
  void* scan_tmp = p;
  p += scan_temp_bytes((int64_t)hist_n);
  p = reinterpret_cast<char*>(((uintptr_t)p + 255) & ~(uintptr_t)255);
  uint64_t* count = reinterpret_cast<uint64_t*>(p);
  p += 64;
  uint32_t* k1 = reinterpret_cast<uint32_t*>(p);
  uint32_t* v1 = k1 + n;
  k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(count), 1,
                              (unsigned long long)n);
  const uint32_t* ki = kin;
  const uint32_t* vi = reinterpret_cast<const uint32_t*>(vin);
  for (int pass = 0; pass < 4; ++pass) {
    // passes alternate between the ping-pong copy and the output
    uint32_t* ko = pass % 2 == 0 ? k1 : kout;
    uint32_t* vo = pass % 2 == 0 ? v1 : reinterpret_cast<uint32_t*>(vout);
    launch_radix_up_pairs(ki, count, (uint64_t)n, 8 * pass, 8, hist, s);
    launch_scan_u32_to_u64(hist, offs, (int64_t)hist_n, scan_tmp, s);
    launch_radix_down_pairs(ki, vi, count, (uint64_t)n, 8 * pass, 8, offs, ko, vo, s);
    ki = ko;
    vi = vo;
  }
  HIPTRY(hipGetLastError(), "sort");
  return PANTHER_OK;
}

}  // namespace

int prepare_bf16(panther_ctx* c, int32_t D, hipStream_t s) {
  PPState* pp = c->pp;
  if (D > kDP) return ctx_fail(c, PANTHER_EINVAL, "the BF16 form supports D <= %d", kDP);
  if (!pp || !c->d_theta || c->theta_D != D)
    return ctx_fail(c, PANTHER_ESTATE, "features for D = %d are not computed", D);
  if (pp->bf16_D == D) return PANTHER_OK;
  pp->bf16_D = 0;
  const int64_t n = c->n;
  // norms as keys, sorted with the vertex ids; then the zero rows past
  // kZeroKeep are dropped and the rest written in that order
  DevBuf keys, tmp;
  int64_t rows = n;
  int rc = ctx_ensure(c, keys, sizeof(uint32_t) * 2 * (size_t)n + sizeof(int32_t) * 2 * (size_t)n + 64,
                      "norm keys");
  if (rc == PANTHER_OK) {
    uint32_t* kin = static_cast<uint32_t*>(keys.p);
    uint32_t* kout = kin + n;
    int32_t* vin = reinterpret_cast<int32_t*>(kout + n);
    int32_t* vout = vin + n;
    unsigned long long* zc = reinterpret_cast<unsigned long long*>(vout + n);  // 16n bytes in
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    k_bf16_norm_keys<<<g, kBlock, 0, s>>>(c->d_theta, c->n, D, (float)c->R, kin, vin);
    rc = hipGetLastError() == hipSuccess ? PANTHER_OK
                                         : ctx_fail(c, PANTHER_EDEVICE, "bf16 norm keys");
    if (rc == PANTHER_OK) rc = sort_pairs(c, tmp, kin, kout, vin, vout, n, s);
    unsigned long long z = 0;
    if (rc == PANTHER_OK) {
      if (hipMemsetAsync(zc, 0, sizeof z, s) != hipSuccess) rc = ctx_fail(c, PANTHER_EDEVICE, "zero rows");
      if (rc == PANTHER_OK) k_count_zero<<<g, kBlock, 0, s>>>(kout, n, zc);
      if (rc == PANTHER_OK && (hipMemcpyAsync(&z, zc, sizeof z, hipMemcpyDeviceToHost, s) != hipSuccess ||
                               hipStreamSynchronize(s) != hipSuccess))
        rc = ctx_fail(c, PANTHER_EDEVICE, "zero rows");
    }
    if (rc == PANTHER_OK) {
      const int64_t zk = std::min<int64_t>((int64_t)z, kZeroKeep);
      const int64_t drop = (int64_t)z - zk;
      rows = n - drop;
      // whole trips of chunks, and one all-padding chunk after them
      const int64_t npad =
          (rows + kTrip * kChunk - 1) / (kTrip * kChunk) * (kTrip * kChunk) + kChunk;
      rc = ctx_ensure(c, pp->b_bf16, sizeof(__bf16) * (size_t)npad * kDP, "bf16 rows");
      if (rc == PANTHER_OK) rc = ctx_ensure(c, pp->b_norm, sizeof(float) * (size_t)npad, "bf16 norms");
      if (rc == PANTHER_OK) rc = ctx_ensure(c, pp->b_sid, sizeof(int32_t) * (size_t)npad, "bf16 row ids");
      if (rc == PANTHER_OK) rc = ctx_ensure(c, pp->b_rank, sizeof(int32_t) * (size_t)n, "bf16 row ranks");
      if (rc == PANTHER_OK) {
        k_bf16_rows_sorted<<<g, kBlock, 0, s>>>(
            c->d_theta, c->n, D, (float)c->R, vout, zk, drop, static_cast<int32_t*>(pp->b_sid.p),
            static_cast<__bf16*>(pp->b_bf16.p), static_cast<float*>(pp->b_norm.p),
            static_cast<int32_t*>(pp->b_rank.p));
        k_bf16_pad_rows<<<(unsigned)((npad - rows + kBlock - 1) / kBlock), kBlock, 0, s>>>(
            rows, npad, static_cast<int32_t*>(pp->b_sid.p), static_cast<__bf16*>(pp->b_bf16.p),
            static_cast<float*>(pp->b_norm.p));
        rc = hipGetLastError() == hipSuccess ? PANTHER_OK
                                             : ctx_fail(c, PANTHER_EDEVICE, "bf16 rows");
      }
    }
    // the scratch is freed only after the kernels that read it are done
    if (hipStreamSynchronize(s) != hipSuccess && rc == PANTHER_OK)
      rc = ctx_fail(c, PANTHER_EDEVICE, "bf16 rows");
  }
  ctx_release(keys);
  ctx_release(tmp);
  TRY(rc);
  pp->bf16_rows = rows;
  TRY(ctx_ensure(c, pp->b_dbmax, 64, "row bounds"));
  HIPTRY(hipMemsetAsync(pp->b_dbmax.p, 0, 64, s), "row bounds");
  k_row_bounds<<<(unsigned)((c->n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
      c->d_theta, c->n, D, (float)c->R, static_cast<unsigned int*>(pp->b_dbmax.p));
  HIPTRY(hipGetLastError(), "row bounds");
  float bounds[2];
  HIPTRY(hipMemcpyAsync(bounds, pp->b_dbmax.p, sizeof bounds, hipMemcpyDeviceToHost, s),
         "row bounds");
  HIPTRY(hipStreamSynchronize(s), "row bounds");
  pp->bf16_err = (double)bounds[1];
  pp->bf16_D = D;
  return PANTHER_OK;
}

namespace panther {

namespace {

// Candidate-pool geometry of a BF16 call with nq queries.
struct PoolGeom {
  int P;          // pool per query
  int cap;        // buffer entries per (query, slice)
  int qw;         // queries per work-group tile
  int64_t tiles;  // query tiles
  int64_t S;      // database slices per tile
};

PoolGeom pool_geom(const panther_ctx* c, int64_t nq, int32_t k, int qw = 0) {
  PoolGeom g{};
  // pool: at least the option and at least 2k (margin for the bfloat16
  // rounding at the pool boundary), a power of two, at most 1024
  g.P = 32;
  while (g.P < c->pp_pool || g.P < 2 * k) g.P <<= 1;
  if (g.P > 1024) g.P = 1024;
  // buffer: P kept keys, at least P more before a compaction is worth its
  // sort, and room for the kCheckEvery chunks between checks
  g.cap = 2 * g.P + kCheckEvery * kChunk;
  // Query tiles of qw queries per work-group: by default 64 for large
  // batches, 32 for medium and 16 for small ones (a tile scans the union of
  // its queries' norm bands, so narrower tiles scan fewer rows; wider ones
  // reuse each row more); the autotuner may choose any of them.  The database is split into
  // slices when the batch has few tiles, so that about two work-groups per
  // CU scan it.
  g.qw = qw ? qw : (nq >= 32768 ? 64 : (nq >= 8192 ? 32 : 16));
  g.tiles = (nq + g.qw - 1) / g.qw;
  const int64_t rows = c->pp && c->pp->bf16_rows ? c->pp->bf16_rows : (int64_t)c->n;
  int64_t S = (2 * (int64_t)c->num_cus + g.tiles - 1) / std::max<int64_t>(g.tiles, 1);
  S = std::max<int64_t>(1, std::min<int64_t>(S, 256));
  S = std::min<int64_t>(S, std::max<int64_t>(1, rows / 4096));
  S = std::min<int64_t>(S, std::max<int64_t>(1, 262144 / g.P));  // bounds the merge work
  g.S = S;
  return g;
}

}  // namespace

// One BF16 call with the pool geometry G: the pool pass, the rerank and the
// exact recompute of the uncertified queries.
static int run_pp_bf16_geom(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq,
                            int32_t D, int32_t k, int32_t* d_ids, double* d_dist, hipStream_t s,
                            const float* qtheta, const PoolGeom& G) {
  PPState* pp = c->pp;
  const int P = G.P, cap = G.cap, qw = G.qw;
  const int64_t tiles = G.tiles, S = G.S;
  const float scale = (float)c->R;
  const size_t buf_bytes = sizeof(uint64_t) * (size_t)nq * S * cap;
  const size_t part_bytes = S > 1 ? sizeof(uint64_t) * (size_t)nq * S * P : 0;
  const size_t ids_bytes = (sizeof(int32_t) + sizeof(float)) * (size_t)nq * P;
  const size_t gtau_bytes = S > 1 ? sizeof(uint64_t) * (size_t)nq : 0;
  TRY(ctx_ensure(c, lane->b_pool, buf_bytes + part_bytes + gtau_bytes + ids_bytes + 256,
                 "pools"));
  TRY(ctx_ensure(c, lane->b_stats, 64, "pp stats"));
  char* base = static_cast<char*>(lane->b_pool.p);
  uint64_t* buf = reinterpret_cast<uint64_t*>(base);
  uint64_t* part = reinterpret_cast<uint64_t*>(base + buf_bytes);
  unsigned long long* gtau =
      S > 1 ? reinterpret_cast<unsigned long long*>(base + buf_bytes + part_bytes) : nullptr;
  int32_t* pool_ids = reinterpret_cast<int32_t*>(base + buf_bytes + part_bytes + gtau_bytes);
  float* pool_d2 = reinterpret_cast<float*>(pool_ids + (size_t)nq * P);
  HIPTRY(hipMemsetAsync(lane->b_stats.p, 0, 64, s), "pp stats");
  const int sort_cap = std::max(cap, P);
  const int64_t rows = pp->bf16_rows;
  const int64_t nchunks = (rows + kTrip * kChunk - 1) / (kTrip * kChunk) * kTrip;
  PoolArgs pa{};
  pa.rows = static_cast<const __bf16*>(pp->b_bf16.p);
  pa.norm = static_cast<const float*>(pp->b_norm.p);
  pa.sid = static_cast<const int32_t*>(pp->b_sid.p);
  pa.rank = static_cast<const int32_t*>(pp->b_rank.p);
  pa.n = (int32_t)rows;
  pa.nchunks = nchunks;
  pa.queries = dq;
  pa.nq = nq;
  pa.P = P;
  pa.cap = cap;
  pa.slices = (int32_t)S;
  pa.sort_cap = sort_cap;
  pa.buf = buf;
  pa.part = part;
  pa.pool_ids = pool_ids;
  pa.pool_d2 = pool_d2;
  pa.q_by_pos = 0;
  pa.exclude_self = 1;
  pa.gtau = gtau;
  pa.stat_products = static_cast<unsigned long long*>(lane->b_stats.p) + 5;
  if (gtau) {
    k_fill_u64<<<(unsigned)((nq + kBlock - 1) / kBlock), kBlock, 0, s>>>(gtau, nq, ~0ull);
    HIPTRY(hipGetLastError(), "pool bounds");
  }
  if (qtheta) {
    TRY(ctx_ensure(c, lane->b_qrows, (sizeof(__bf16) * kDP + sizeof(float)) * (size_t)nq,
                   "query bf16 rows"));
    __bf16* qr = static_cast<__bf16*>(lane->b_qrows.p);
    float* qn = reinterpret_cast<float*>(qr + (size_t)nq * kDP);
    k_bf16_query_rows<<<(unsigned)((nq + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        qtheta, D, dq, nq, scale, qr, qn);
    HIPTRY(hipGetLastError(), "query bf16 rows");
    pa.qrows = qr;
    pa.qnorm = qn;
    pa.q_by_pos = 1;
    pa.exclude_self = 0;
  }
  // query positions in ascending order of operand norm (tiles of similar
  // norms keep their bands narrow)
  {
    const size_t half = ((size_t)nq + 63) / 64 * 64;
    TRY(ctx_ensure(c, lane->b_qsort, (2 * sizeof(uint32_t) + 2 * sizeof(int32_t)) * half,
                   "query order"));
    uint32_t* kin = static_cast<uint32_t*>(lane->b_qsort.p);
    uint32_t* kout = kin + half;
    int32_t* vin = reinterpret_cast<int32_t*>(kout + half);
    int32_t* vout = vin + half;
    k_query_norm_keys<<<(unsigned)((nq + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        pa.norm, pa.rank, pa.qnorm, dq, nq, kin, vin);
    HIPTRY(hipGetLastError(), "query order");
    TRY(sort_pairs(c, lane->b_qsort_tmp, kin, kout, vin, vout, nq, s));
    pa.q_order = vout;
  }
  const size_t sort_lds = sizeof(uint64_t) * (size_t)sort_cap * (kBlock / kWave);
  const void* pool_fn = qw == 64   ? (const void*)k_pp_pool<64>
                        : qw == 32 ? (const void*)k_pp_pool<32>
                                   : (const void*)k_pp_pool<16>;
  HIPTRY(hipFuncSetAttribute(pool_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sort_lds),
         "pp pool attribute");
  auto launch_pool = [&](const PoolArgs& args, unsigned gy) {
    if (qw == 64)
      k_pp_pool<64><<<dim3((unsigned)tiles, gy), kBlock, sort_lds, s>>>(args);
    else if (qw == 32)
      k_pp_pool<32><<<dim3((unsigned)tiles, gy), kBlock, sort_lds, s>>>(args);
    else
      k_pp_pool<16><<<dim3((unsigned)tiles, gy), kBlock, sort_lds, s>>>(args);
  };
  if (S > 1) {
    // bound pass: one work-group per tile scans the kBoundChunks chunks
    // nearest its median norm and publishes each query's P-th key, so that
    // the slices start from a tight bound instead of each filling its own
    // pool from the first rows
    PoolArgs pb = pa;
    pb.slices = 1;
    pb.max_chunks = kBoundChunks;
    pb.bound_only = 1;
    launch_pool(pb, 1u);
    HIPTRY(hipGetLastError(), "pp pool bound");
  }
  launch_pool(pa, (unsigned)S);
  HIPTRY(hipGetLastError(), "pp pool");
  if (S > 1) {
    k_pp_merge<<<(unsigned)nq, kBlock, 0, s>>>(pa);
    HIPTRY(hipGetLastError(), "pp merge");
  }
  unsigned long long* st = static_cast<unsigned long long*>(lane->b_stats.p);
  TRY(ctx_ensure(c, lane->b_fb, (2 * sizeof(int32_t) + sizeof(double)) * (size_t)nq,
                 "uncertified queries"));
  int32_t* fb_list = static_cast<int32_t*>(lane->b_fb.p);
  double* fb_tau_d = reinterpret_cast<double*>(fb_list + ((size_t)nq + 1) / 2 * 2);
  int32_t* fb_tau_v = reinterpret_cast<int32_t*>(fb_tau_d + nq);
  RerankArgs ra{};
  ra.theta = c->d_theta;
  ra.db_max = static_cast<const float*>(pp->b_dbmax.p);
  ra.scale = (double)scale;
  ra.fb_list = fb_list;
  ra.fb_tau_d = fb_tau_d;
  ra.fb_tau_v = fb_tau_v;
  ra.fb_n = st + 3;
  ra.force = c->pp_recompute_all;
  ra.qtheta = qtheta ? qtheta : c->d_theta;
  ra.D = D;
  ra.queries = dq;
  ra.nq = nq;
  ra.P = P;
  ra.k = k;
  ra.pool_ids = pool_ids;
  ra.pool_d2 = pool_d2;
  ra.inv_s2 = 1.0f / (scale * scale);
  ra.out_ids = d_ids;
  ra.out_dist = d_dist;
  ra.stat_hits = st;
  ra.stat_err = st + 1;
  ra.stat_ret = st + 2;
  const size_t rr_lds = rerank_lds(P);
  HIPTRY(hipFuncSetAttribute((const void*)k_pp_rerank, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)rr_lds),
         "pp rerank attribute");
  k_pp_rerank<<<(unsigned)nq, kBlock, rr_lds, s>>>(ra);
  HIPTRY(hipGetLastError(), "pp rerank");
  unsigned long long hs[6];
  HIPTRY(hipMemcpyAsync(hs, st, sizeof hs, hipMemcpyDeviceToHost, s), "pp stats");
  HIPTRY(hipStreamSynchronize(s), "pp stats");
  // queries whose pool boundary is not certified: exact recompute
  if (hs[3] > 0) {
    TRY(ctx_ensure(c, lane->b_fbw, knn_range_bytes((int64_t)hs[3]), "exact recompute"));
    // the norm-ordered BF16 rows bound each query's candidates (a dropped
    // zero row is never needed: the kept zero rows of smaller id tie it)
    KnnBand kb{static_cast<const float*>(pp->b_norm.p), static_cast<const int32_t*>(pp->b_sid.p),
               pp->bf16_rows, (double)scale, pp->bf16_err};
    const int e = launch_knn_recompute(c->d_theta, c->n, D, qtheta ? qtheta : c->d_theta, !qtheta,
                                       dq, fb_list, (int64_t)hs[3], fb_tau_d, fb_tau_v, k,
                                       c->num_cus, lane->b_fbw.p, st + 4, d_ids, d_dist, s,
                                       c->pp_recompute_all == 2 ? (uint32_t)(k - 1) : ~0u, &kb);
    HIPTRY((hipError_t)e, "pp exact recompute");
    HIPTRY(hipStreamSynchronize(s), "pp exact recompute");
  }
  lane->have_stats = true;
  lane->mean_pre_recall = hs[2] ? (double)hs[0] / (double)hs[2] : 1.0;
  double e;
  std::memcpy(&e, &hs[1], sizeof e);
  lane->max_rel_err = e;
  lane->stat_nq = nq;
  lane->stat_fallback = (int64_t)hs[3];
  lane->stat_scanned = (double)hs[5] / ((double)nq * (double)c->n);
  return PANTHER_OK;
}

// The pool tile width of a BF16 call: forced by "pp.qw", else the tuned
// choice of its shape class (rows, D, batch size and k rounded to powers of
// two, pool, cross-graph), else, when autotuning, timed now on the main lane
// (each width warmed once and timed once; the answer is the same for
// either, since the exact rerank decides it), else the default.
static int pool_width(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, int32_t D,
                      int32_t k, int32_t* d_ids, double* d_dist, hipStream_t s,
                      const float* qtheta, int* qw_out) {
  *qw_out = c->pp_qw;
  if (c->pp_qw) return PANTHER_OK;
  int nq_bucket = 0;
  while ((int64_t(2) << nq_bucket) <= nq) ++nq_bucket;
  int k_bucket = 1;
  while (k_bucket < k) k_bucket <<= 1;
  char key[256];
  snprintf(key, sizeof key, "gfx950:pp:rows%lld:D%d:nq2^%d:k%d:P%d:cu%d:x%d",
           (long long)c->pp->bf16_rows, D, nq_bucket, k_bucket, pool_geom(c, nq, k).P,
           c->num_cus, qtheta ? 1 : 0);
  {
    std::lock_guard<std::mutex> g(c->pp_tune_mu);
    auto it = c->pp_qw_tuned.find(key);
    if (it != c->pp_qw_tuned.end()) {
      *qw_out = it->second;
      return PANTHER_OK;
    }
  }
  int qw = 0;
  for (const std::vector<int>& f : tune_cache_read(key))
    if (f.size() == 1 && (f[0] == 16 || f[0] == 32 || f[0] == 64)) qw = f[0];
  if (!qw && c->autotune && nq >= 2048 && lane == &c->lane0) {
    hipEvent_t e0, e1;
    HIPTRY(hipEventCreate(&e0), "pp autotune");
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return ctx_fail(c, PANTHER_EDEVICE, "pp autotune: event");
    }
    float best = 1e30f;
    int st = PANTHER_OK;
    for (int w : {16, 32, 64}) {
      const PoolGeom G = pool_geom(c, nq, k, w);
      if (!st) st = run_pp_bf16_geom(c, lane, dq, nq, D, k, d_ids, d_dist, s, qtheta, G);
      if (!st) st = ctx_hip(c, hipEventRecord(e0, s), "pp autotune");
      if (!st) st = run_pp_bf16_geom(c, lane, dq, nq, D, k, d_ids, d_dist, s, qtheta, G);
      if (!st) st = ctx_hip(c, hipEventRecord(e1, s), "pp autotune");
      if (!st) st = ctx_hip(c, hipEventSynchronize(e1), "pp autotune");
      float ms = 0.f;
      if (!st) st = ctx_hip(c, hipEventElapsedTime(&ms, e0, e1), "pp autotune");
      if (!st && ms < best) {
        best = ms;
        qw = w;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    tune_cache_append(key, {qw});
  }
  if (qw) {
    std::lock_guard<std::mutex> g(c->pp_tune_mu);
    c->pp_qw_tuned[key] = qw;
  }
  *qw_out = qw;
  return PANTHER_OK;
}

// Pool pass + rerank over the database context c.  qtheta (null: c's own
// features) holds the queries' feature rows when they come from another
// graph; their bf16 operands are then gathered per query first.
int run_pp_bf16(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, int32_t D, int32_t k,
                int32_t* d_ids, double* d_dist, hipStream_t s, const float* qtheta) {
  PPState* pp = c->pp;
  if (D > kDP) return ctx_fail(c, PANTHER_EINVAL, "the BF16 form supports D <= %d", kDP);
  if (!pp || pp->bf16_D != D) return ctx_fail(c, PANTHER_ESTATE, "bf16 rows not prepared");
  int qw = 0;
  TRY(pool_width(c, lane, dq, nq, D, k, d_ids, d_dist, s, qtheta, &qw));
  return run_pp_bf16_geom(c, lane, dq, nq, D, k, d_ids, d_dist, s, qtheta, pool_geom(c, nq, k, qw));
}

}  // namespace panther

// Device bytes of the lane scratch a BF16 call of nq queries takes (the
// FP64 form takes none): pools, statistics, query order and its sort,
// certificate, exact recompute of every query, cross-graph query rows.
size_t pp_lane_bytes(const panther_ctx* c, int64_t nq, int32_t k) {
  if (nq <= 0) return 0;
  if (c->pp_form == PANTHER_PP_FP64) return 0;
  const size_t n = (size_t)nq;
  // either tile width may be chosen: the larger need
  size_t b = 0;
  for (int w : {16, 32, 64}) {
    const panther::PoolGeom G = panther::pool_geom(c, nq, k, w);
    b = std::max(b, sizeof(uint64_t) * n * G.S * G.cap + sizeof(uint64_t) * n +
                        (G.S > 1 ? sizeof(uint64_t) * n * G.S * G.P : 0) +
                        (sizeof(int32_t) + sizeof(float)) * n * G.P + 256);
  }
  b += 64;
  b += (2 * sizeof(uint32_t) + 2 * sizeof(int32_t)) * ((n + 63) / 64 * 64);
  b += sort_pairs_bytes(nq);
  b += (2 * sizeof(int32_t) + sizeof(double)) * n;
  b += panther::knn_range_bytes(nq);
  b += (sizeof(uint16_t) * 64 + sizeof(float)) * n;
  return b;
}
