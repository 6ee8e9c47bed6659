// Host-side launchers of the Panther kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace panther {

// Per-vertex record read by the walk: CSR row start, degree, and the row's
// weight sum W_v split in two 32-bit halves (one 16-byte load per step).
struct VRec {
  int32_t start;
  int32_t deg;
  uint32_t w_lo;
  uint32_t w_hi;
};

// ---- prep (graph load) ----
// Validation: sets bit 0 of *err for a decreasing row_ptr, bit 1 for a
// column out of range.
void launch_validate(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                     uint32_t* err, hipStream_t s);
// Symmetry (column ids already validated): sets bit 2 of *err when some
// entry v->u of weight w has no matching u->v of weight w (multiplicities
// compared).  sorted: n bytes of scratch.
void launch_check_symmetric(const int32_t* row_ptr, const int32_t* col, const uint32_t* w,
                            int32_t n, uint8_t* sorted, uint32_t* err, hipStream_t s);
// Row sums into vrec; rows longer than 256 entries go to big_rows.
void launch_rowsum(const int32_t* row_ptr, const uint32_t* w, int32_t n, VRec* vrec,
                   uint64_t* max_w, int32_t* big_rows, uint32_t* n_big, hipStream_t s);
void launch_rowsum_big(const int32_t* big_rows, uint32_t n_big, const uint32_t* w, VRec* vrec,
                       uint64_t* max_w, hipStream_t s);
// Start-set flags (1 where W_v > 0, or everywhere when start_all).
void launch_start_flags(const VRec* vrec, int32_t n, int start_all, uint32_t* flags,
                        hipStream_t s);
void launch_start_scatter(const uint32_t* flags, const uint64_t* pos, int32_t n, int32_t* vstart,
                          hipStream_t s);
// Inclusive per-row weight prefixes (uint32 when every W_v < 2^32).
void launch_prefix32(const VRec* vrec, const uint32_t* w, int32_t n, const int32_t* big_rows,
                     uint32_t n_big, uint32_t* pfx, hipStream_t s);
void launch_prefix64(const VRec* vrec, const uint32_t* w, int32_t n, const int32_t* big_rows,
                     uint32_t n_big, uint64_t* pfx, hipStream_t s);

// Walk acceleration for 32-bit prefixes: edge[e] = {prefix, column} and the
// per-row guide table (entry b = first edge any draw of bucket b can pick).
void launch_pack_edges(const uint32_t* pfx, const int32_t* col, int64_t m, uint2* edge,
                       hipStream_t s);
void launch_guide(const VRec* vrec, const uint32_t* pfx, int32_t n, const int32_t* big_rows,
                  uint32_t n_big, int32_t* guide, hipStream_t s);

// 64-byte fat guide records (4 x uint4 per bucket), see prep.hip.
void launch_fat_guide(const VRec* vrec, const uint32_t* pfx, const int32_t* col,
                      const int32_t* guide, int32_t n, const int32_t* big_rows, uint32_t n_big,
                      uint4* fat, hipStream_t s);

// {vertex, row start, degree, W} per start-set entry (32-bit weight sums).
void launch_start_records(const int32_t* vstart, int32_t nstart, const VRec* vrec, int4* out,
                          hipStream_t s);

// ---- device-wide exclusive scan: out[i] = sum in[0..i), out[n] = total ----
size_t scan_temp_bytes(int64_t n);
void launch_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, void* temp,
                            hipStream_t s);

// ---- walk ----
// 64-bit prefixes: bisection over pfx64 + col.  32-bit prefixes: guide
// table + packed edge records.
void launch_walk64(int stride, const VRec* vrec, const uint64_t* pfx, const int32_t* col,
                   const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                   int32_t* paths, hipStream_t s);
void launch_walk32(int stride, const VRec* vrec, const uint2* edge, const uint4* fat,
                   const int4* start_rec, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                   int32_t* paths, hipStream_t s);

// ---- index by stable LSD radix sort of (vertex, path id) pairs ----
constexpr int kRadixPassBits = 8;
uint64_t radix_tiles_paths(uint64_t R, int T);
uint64_t radix_tiles_pairs(uint64_t nnz);
// hist: [256][tiles] digit-major histograms of the pass
void launch_radix_up_paths(int stride, const int32_t* paths, uint64_t R, int T, int shift,
                           int bits, uint32_t* hist, hipStream_t s);
void launch_radix_down_paths(int stride, const int32_t* paths, uint64_t R, int T, int shift,
                             int bits, const uint64_t* offsets, uint32_t* key_out,
                             uint32_t* val_out, hipStream_t s);
// pair passes: the pair count is read on the device (nnz_dev); grids are
// sized for nnz_cap >= nnz
void launch_radix_up_pairs(const uint32_t* keys, const uint64_t* nnz_dev, uint64_t nnz_cap,
                           int shift, int bits, uint32_t* hist, hipStream_t s);
void launch_radix_down_pairs(const uint32_t* keys, const uint32_t* vals, const uint64_t* nnz_dev,
                             uint64_t nnz_cap, int shift, int bits, const uint64_t* offsets,
                             uint32_t* key_out, uint32_t* val_out, hipStream_t s);
void launch_copy_u64(const uint64_t* src, uint64_t* dst, hipStream_t s);
void launch_list_bounds(const uint32_t* keys, const uint64_t* nnz_dev, uint64_t nnz_cap, int32_t n,
                        uint64_t* inv_ptr, hipStream_t s);

// ---- count + top-k, plain form: one launch per query ----
struct TopkScratch {
  uint32_t* cnt;       // dense counters [n], zero between queries
  int32_t* touched;    // [n]
  uint32_t* ctl;       // [4]: touched count, ticket, spare
};
// qp: the query id in device memory (an id outside [0, n) yields a padded
// row with out_len -1); list_len sizes the grid (any value is correct).
void launch_topk_plain(int stride, const int32_t* qp, int32_t n, const uint64_t* inv_ptr,
                       const uint32_t* inv_pid, const int32_t* paths, uint64_t list_len,
                       TopkScratch sc, int32_t k, int32_t* out_ids, uint32_t* out_counts,
                       int32_t* out_len, hipStream_t s);

void launch_iota(int32_t* out, int32_t n, hipStream_t s);
// p[0, n) = 0 with a kernel (capturable, unlike a memset node)
void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s);
void launch_query_lengths(const uint64_t* inv_ptr, const int32_t* queries, int64_t nq,
                          uint64_t* out, hipStream_t s);

// A norm-ordered copy of a kNN database: rows p < rows in ascending order
// of their stored squared norm norm_s[p] (units scaled by scale), vertex
// sid[p]; err bounds the distance between a stored row and scale * theta_v.
struct KnnBand {
  const float* norm_s;
  const int32_t* sid;
  int64_t rows;
  double scale;
  double err;
};

// Exact recompute of listed queries from a known bound (knn.hip): rows[i]
// (i < nr) names the output row of query queries[rows[i]], and (tau_d[i],
// tau_v[i]) is an exact (d2, id) pair that at least k rows reach.  work:
// device memory of knn_range_bytes(nr) bytes.  band (required): each
// query scans only its norm band of that copy, whose rows must include
// every candidate.  A list keeps up to min(cap, 4096) candidates; lists
// that outgrow it are recomputed by the full brute force.
size_t knn_range_bytes(int64_t nr);
int launch_knn_recompute(const float* theta, int32_t n, int32_t D, const float* qtheta,
                         bool exclude_self, const int32_t* queries, const int32_t* rows,
                         int64_t nr, const double* tau_d, const int32_t* tau_v, int32_t k,
                         int num_cus, void* work, unsigned long long* ov_n_dev,
                         int32_t* out_ids, double* out_dist, hipStream_t s, uint32_t cap,
                         const KnnBand* band);

}  // namespace panther
