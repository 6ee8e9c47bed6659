// Host runtime state of a Panther context (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

struct BatchState;

// Device buffer that keeps its allocation across calls and grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Page-locked host memory (staging of plans and query lengths).
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Panther++ data shared by every lane: bf16 copy of theta and its norms.
struct PPState {
  DevBuf b_bf16, b_norm, b_iota;
  DevBuf b_sid, b_rank;  // BF16 rows in norm order: original id per row, row per id
  DevBuf b_dbmax;  // float: an upper bound on max_v |theta_v| (Euclidean)
  int32_t bf16_D = 0;
  int64_t bf16_rows = 0;  // rows of the norm-ordered BF16 database
  double bf16_err = 0.0;  // >= max over rows of |bf16 row - theta_v * R|
};

// Scratch of one query stream.  The context's own calls use lane 0; the
// serving loop runs several lanes concurrently, each on its own stream,
// over the same read-only graph, paths, index and features.
struct Lane {
  BatchState* batch = nullptr;
  DevBuf b_qlen, b_pool, b_out, b_stats, b_q, b_qrows, b_fb, b_fbw, b_qsort, b_qsort_tmp;
  int64_t stat_nq = 0;        // queries of the last BF16-form call
  int64_t stat_fallback = 0;  // of them, recomputed exactly (boundary not certified)
  double stat_scanned = 0.0;  // (query, row) products of its pool pass / (queries * vertices)
  PinnedBuf h_qlen;  // path-list lengths of the last call's queries
  bool have_stats = false;
  double max_rel_err = 0.0;
  double mean_pre_recall = 0.0;
};

struct panther_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::mutex err_mu;
  int num_cus = 256;
  int lds_per_block = 65536;
  // options
  int topk_form = 1;  // PANTHER_FORM_BATCHED
  int pp_form = 1;    // PANTHER_PP_BF16
  int pp_pool = 256;
  int pp_recompute_all = 0;  // test: recompute every full-pool query (2: via brute force)
  int pp_qw = 0;             // BF16 pool tile width (0: tuned)
  int autotune = 1;
  std::map<std::string, int> pp_qw_tuned;  // tuned pool tile width per shape class
  std::mutex pp_tune_mu;
  int64_t fail_alloc_after = -1;
  std::mutex alloc_mu;
  // graph
  bool has_graph = false;
  int32_t n = 0;
  int64_t m = 0;
  int32_t* d_col = nullptr;
  panther::VRec* d_vrec = nullptr;
  void* d_pfx = nullptr;
  bool pfx64 = false;
  uint2* d_edge = nullptr;    // {prefix, column} when every W_v < 2^32
  uint4* d_fat = nullptr;     // 64-byte guide records, same case
  int4* d_start_rec = nullptr;  // {v, row start, degree, W} per start entry, same case
  int32_t* d_vstart = nullptr;
  int32_t nstart = 0;
  uint64_t max_w = 0;
  // paths + index
  bool has_paths = false;
  int32_t T = 0;
  int64_t R = 0;
  uint64_t seed = 0;
  int stride = 0;
  int32_t* d_paths = nullptr;
  uint64_t* d_inv_ptr = nullptr;
  uint32_t* d_inv_pid = nullptr;
  int64_t nnz = 0;
  // storage reused across sample_paths / query calls
  DevBuf b_paths, b_inv_pid, b_inv_ptr, b_keys0, b_keys1, b_vtmp, b_hist, b_offs, b_stemp, b_nnz;
  DevBuf b_allv;  // vertex ids 0..n-1 (all-vertex top-k)
  DevBuf b_queries, b_outs;
  // dense query scratch (plain form, hub queries)
  uint32_t* d_cnt = nullptr;
  int32_t* d_touched = nullptr;
  uint32_t* d_ctl = nullptr;
  // scratch of the context's own query calls
  Lane lane0;
  // calls on different streams share the scratch above: each call waits
  // for the previous one's completion event before using it
  hipEvent_t order_ev = nullptr;
  bool order_pending = false;
  // stage timing (option "timing")
  int timing = 0;
  hipEvent_t ev[10] = {};
  bool ev_used[5] = {};
  // Panther++
  float* d_theta = nullptr;
  int32_t theta_D = 0;
  PPState* pp = nullptr;
};

#define TRY(expr)                      \
  do {                                 \
    int _st = (expr);                  \
    if (_st != PANTHER_OK) return _st; \
  } while (0)
#define HIPTRY(expr, what) TRY(ctx_hip(c, (expr), what))

int ctx_fail(panther_ctx* c, int code, const char* fmt, ...);
int ctx_hip(panther_ctx* c, hipError_t e, const char* what);
int ctx_alloc(panther_ctx* c, void** p, size_t bytes, const char* what);  // thread-safe
// Makes b hold at least `bytes`; the contents are not preserved on growth.
int ctx_ensure(panther_ctx* c, DevBuf& b, size_t bytes, const char* what);
void ctx_release(DevBuf& b);
int pinned_ensure(panther_ctx* c, PinnedBuf& b, size_t bytes, const char* what);
void pinned_release(PinnedBuf& b);
// Path-list lengths of the queries, gathered on the device into the lane's
// b_qlen and, with to_host, copied back to its pinned buffer (*len points
// there until the lane's next call; nullptr without to_host).
int query_lengths(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, hipStream_t s,
                  const uint64_t** len, bool to_host = true);
void ctx_free(void* p);
// Stage timing: stage i is bracketed by events 2i and 2i+1.
void stage_begin(panther_ctx* c, int stage, hipStream_t s);
void stage_end(panther_ctx* c, int stage, hipStream_t s);
int order_begin(panther_ctx* c, hipStream_t s);
int order_end(panther_ctx* c, hipStream_t s);
int stage_queries(panther_ctx* c, const int32_t* queries, int64_t nq, int mem, hipStream_t s,
                  std::vector<int32_t>& hq, const int32_t** dq, void** dq_owned);

// batched form (batch.hip).  With theta != nullptr the pass writes Panther++
// feature rows (k = D) instead of ids/counts.
// Enqueues the work on s; returns without waiting for it.  qlen are the
// lengths on the host, or nullptr for a batch that batched_plan_on_device
// accepts: it is then planned from the lane's device lengths (b_qlen).
bool batched_plan_on_device(int64_t nq);
// Autotuner cache (a text file, flock-guarded): the integer fields of every
// line of `key`, in file order; appending adds one line.
std::vector<std::vector<int>> tune_cache_read(const std::string& key);
void tune_cache_append(const std::string& key, const std::vector<int>& fields);
int run_batched(panther_ctx* c, Lane* lane, const int32_t* dq, const uint64_t* qlen, int64_t nq,
                int32_t k, int32_t* d_ids, uint32_t* d_counts, int32_t* d_len, float* theta,
                hipStream_t s);
int set_batch_option(panther_ctx* c, const std::string& key, int64_t value);
// copies the forced batch options of lane 0 to another lane
void copy_batch_options(panther_ctx* c, Lane* dst);
void free_batch_state(Lane* lane);
// drops the lane's captured graph and its repeat detection (new paths)
void forget_batch_graph(Lane* lane);
void free_lane(Lane* lane);
// Memory accounting of the serving loop's admission: the lane's tier and
// bucket limits (taken while the lane is idle), an upper bound on the device
// bytes a query with path-list length L adds to a batched call of that lane
// (k <= kmax), the call's fixed bytes, and what a lane holds now.
struct BatchSizing {
  uint64_t T;
  uint64_t LB;       // longest list counted in one work-group's LDS table
  int hub_bits_max;  // largest log2 bucket count of a hub query
  int bucket_bias;   // extra log2 buckets per hub query
};
BatchSizing batched_sizing(panther_ctx* c, Lane* lane);
size_t batched_query_bytes(const BatchSizing& z, uint64_t L, int32_t kmax);
size_t batched_fixed_bytes();
size_t lane_device_bytes(const Lane* lane);
// Device bytes of the lane scratch a Panther++ call of nq queries uses
// (k <= kmax), in the context's current form.
size_t pp_lane_bytes(const panther_ctx* c, int64_t nq, int32_t kmax);

// Panther++ (pp.hip, knn.hip, pp_bf16.hip)
void free_pp_state(panther_ctx* c);
int ensure_features(panther_ctx* c, int32_t D, hipStream_t s);
// bf16 rows for the precision form (shared by lanes; call before lanes run)
int prepare_bf16(panther_ctx* c, int32_t D, hipStream_t s);
// Panther++ top-k for device queries into device outputs on one lane
int run_pp(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, int32_t D, int32_t k,
           int32_t* d_ids, double* d_dist, hipStream_t s);
