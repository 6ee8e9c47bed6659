// Batched form of the Panther query (placeholder: routes through the plain
// kernels until the persistent kernel lands).
#include "../../include/panther.h"
#include "runtime.h"

using namespace panther;

int run_topk_batched(panther_ctx* c, const int32_t* dq, const std::vector<int32_t>& hq,
                     int64_t nq, int32_t k, int32_t* d_ids, uint32_t* d_counts, int32_t* d_len,
                     hipStream_t s) {
  (void)dq;
  TopkScratch sc{c->d_cnt, c->d_touched, c->d_ctl};
  for (int64_t i = 0; i < nq; ++i) {
    const int32_t q = hq[i];
    launch_topk_plain(c->stride, q, c->d_inv_ptr, c->d_inv_pid, c->d_paths,
                      c->h_inv_ptr[q + 1] - c->h_inv_ptr[q], sc, k, d_ids + i * k,
                      d_counts + i * k, d_len + i, s);
  }
  return ctx_hip(c, hipGetLastError(), "topk batched");
}

int set_batch_option(panther_ctx* c, const std::string& key, int64_t value) {
  (void)value;
  return ctx_fail(c, PANTHER_EINVAL, "unknown option '%s'", key.c_str());
}

void free_batch_state(panther_ctx* c) { (void)c; }
