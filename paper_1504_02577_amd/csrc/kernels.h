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

// ---- device-wide exclusive scan: out[i] = sum in[0..i), out[n] = total ----
size_t scan_temp_bytes(int64_t n);
void launch_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, void* temp,
                            hipStream_t s);

// ---- walk ----
void launch_walk(int stride, bool pfx64, const VRec* vrec, const void* pfx, const int32_t* col,
                 const int32_t* vstart, int32_t nstart, int32_t T, uint64_t R, uint64_t seed,
                 int32_t* paths, hipStream_t s);

// ---- index ----
void launch_index_count(int stride, const int32_t* paths, uint64_t R, uint32_t* cnt,
                        hipStream_t s);
void launch_index_scatter(int stride, const int32_t* paths, uint64_t R,
                          unsigned long long* cursor, uint32_t* inv_pid, hipStream_t s);
// Classifies lists by length: lengths 2..64 sorted by one wave each (in the
// classification kernel's sibling), 65..4096 listed in mid, >4096 in big.
void launch_seg_sort_small(const uint64_t* inv_ptr, int32_t n, uint32_t* inv_pid,
                           int32_t* mid, uint32_t* n_mid, int32_t* big, uint32_t* n_big,
                           hipStream_t s);
void launch_seg_sort_mid(const uint64_t* inv_ptr, const int32_t* mid, uint32_t n_mid,
                         uint32_t* inv_pid, hipStream_t s);
// Big lists: chunk sort (4096) then merge passes; descs are per-block
// (list start, list length, block offset) triples prepared by the host.
struct SegBlock {
  uint64_t start;
  uint32_t len;
  uint32_t off;  // first element (sort) / output position (merge) of the block
};
void launch_seg_chunk_sort(const SegBlock* blocks, uint32_t nblocks, uint32_t* data,
                           hipStream_t s);
void launch_seg_merge(const SegBlock* blocks, uint32_t nblocks, uint32_t width,
                      const uint32_t* src, uint32_t* dst, hipStream_t s);
void launch_seg_copy(const SegBlock* blocks, uint32_t nblocks, const uint32_t* src,
                     uint32_t* dst, hipStream_t s);

// ---- count + top-k, plain form: one launch per query ----
struct TopkScratch {
  uint32_t* cnt;       // dense counters [n], zero between queries
  int32_t* touched;    // [n]
  uint32_t* ctl;       // [4]: touched count, ticket, spare
};
void launch_topk_plain(int stride, int32_t q, const uint64_t* inv_ptr, const uint32_t* inv_pid,
                       const int32_t* paths, uint64_t list_len, TopkScratch sc, int32_t k,
                       int32_t* out_ids, uint32_t* out_counts, int32_t* out_len,
                       hipStream_t s);

}  // namespace panther
