// Panther++ (Sec. 3.3, Algorithm 2): feature vectors and nearest-neighbour
// queries behind the C ABI.
//
// theta(v) = the D largest similarities c(v, u) / R over u != v, descending,
// zero-padded, in single precision.  It is the batched top-k pass run over
// every vertex with k = D, writing count / R instead of (id, count).
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/panther.h"
#include "common.h"
#include "runtime.h"

using namespace panther;

namespace panther {
size_t knn_fp64_lds(int D);
int launch_knn_fp64(const float* theta, int32_t n, int32_t D, const float* qtheta,
                    bool exclude_self, const int32_t* queries, const int32_t* rows, int64_t nq,
                    int32_t k, int32_t* out_ids, double* out_dist, hipStream_t s);
int run_pp_bf16(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, int32_t D, int32_t k,
                int32_t* d_ids, double* d_dist, hipStream_t s, const float* qtheta);
}  // namespace panther

namespace {

__global__ void k_iota(int32_t* out, int32_t n) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = i;
}

}  // namespace

void free_pp_state(panther_ctx* c) {
  c->lane0.have_stats = false;
  if (!c->pp) return;
  for (DevBuf* b : {&c->pp->b_bf16, &c->pp->b_norm, &c->pp->b_iota, &c->pp->b_dbmax,
                    &c->pp->b_sid, &c->pp->b_rank})
    ctx_release(*b);
  delete c->pp;
  c->pp = nullptr;
}

static PPState* pp_state(panther_ctx* c) {
  if (!c->pp) c->pp = new PPState();
  return c->pp;
}

// Computes theta for dimension D unless it is already there.
int ensure_features(panther_ctx* c, int32_t D, hipStream_t s) {
  if (c->d_theta && c->theta_D == D) return PANTHER_OK;
  PPState* pp = pp_state(c);
  ctx_free(c->d_theta);
  c->d_theta = nullptr;
  c->theta_D = 0;
  pp->bf16_D = 0;
  void* p;
  TRY(ctx_alloc(c, &p, sizeof(float) * (size_t)c->n * (size_t)D, "features"));
  c->d_theta = static_cast<float*>(p);
  TRY(ctx_ensure(c, pp->b_iota, sizeof(int32_t) * (size_t)c->n, "vertex ids"));
  int32_t* ids = static_cast<int32_t*>(pp->b_iota.p);
  k_iota<<<(unsigned)((c->n + 255) / 256), 256, 0, s>>>(ids, c->n);
  HIPTRY(hipGetLastError(), "features");
  const uint64_t* qlen = nullptr;
  TRY(query_lengths(c, &c->lane0, ids, c->n, s, &qlen, !batched_plan_on_device(c->n)));
  stage_begin(c, 3, s);
  TRY(run_batched(c, &c->lane0, ids, qlen, c->n, D, nullptr, nullptr, nullptr, c->d_theta, s));
  stage_end(c, 3, s);
  c->theta_D = D;
  return PANTHER_OK;
}

extern "C" int panther_get_features(panther_ctx* c, int32_t D, float* out, int mem) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "get_features before sample_paths");
  if (D < 1 || D > 256) return ctx_fail(c, PANTHER_EINVAL, "D must lie in [1, 256]");
  if (!out) return ctx_fail(c, PANTHER_EINVAL, "null output");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  TRY(order_begin(c, c->stream));
  TRY(ensure_features(c, D, c->stream));
  HIPTRY(hipMemcpyAsync(out, c->d_theta, sizeof(float) * (size_t)c->n * D,
                        mem == PANTHER_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                  : hipMemcpyDeviceToHost,
                        c->stream),
         "get_features");
  TRY(order_end(c, c->stream));
  HIPTRY(hipStreamSynchronize(c->stream), "get_features");
  return PANTHER_OK;
}

extern "C" int panther_pp_topk(panther_ctx* c, const int32_t* queries, int64_t nq, int32_t D,
                               int32_t k, int32_t* out_ids, double* out_dist, int mem,
                               void* stream) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "pp_topk before sample_paths");
  if (D < 1 || D > 256) return ctx_fail(c, PANTHER_EINVAL, "D must lie in [1, 256]");
  if (k < 1 || k > 256) return ctx_fail(c, PANTHER_EINVAL, "k must lie in [1, 256]");
  if (nq < 0) return ctx_fail(c, PANTHER_EINVAL, "nq must be >= 0");
  if (mem != PANTHER_MEM_HOST && mem != PANTHER_MEM_DEVICE)
    return ctx_fail(c, PANTHER_EINVAL, "bad mem");
  if (nq == 0) return PANTHER_OK;
  if (!queries || !out_ids || !out_dist) return ctx_fail(c, PANTHER_EINVAL, "null buffer");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::vector<int32_t> hq;
  const int32_t* dq = nullptr;
  void* owned = nullptr;
  int st = stage_queries(c, queries, nq, mem, s, hq, &dq, &owned);
  struct Own {
    void* p;
    ~Own() { ctx_free(p); }
  } own{owned};
  if (st) return st;
  TRY(order_begin(c, s));
  TRY(ensure_features(c, D, s));
  if (c->pp_form == PANTHER_PP_BF16) TRY(prepare_bf16(c, D, s));
  Lane* lane = &c->lane0;
  int32_t* d_ids = out_ids;
  double* d_dist = out_dist;
  if (mem == PANTHER_MEM_HOST) {
    TRY(ctx_ensure(c, lane->b_out, (sizeof(int32_t) + sizeof(double)) * (size_t)nq * k,
                   "pp outputs"));
    d_dist = static_cast<double*>(lane->b_out.p);
    d_ids = reinterpret_cast<int32_t*>(d_dist + (size_t)nq * k);
  }
  stage_begin(c, 4, s);
  TRY(run_pp(c, lane, dq, nq, D, k, d_ids, d_dist, s));
  stage_end(c, 4, s);
  TRY(order_end(c, s));
  if (mem == PANTHER_MEM_HOST) {
    HIPTRY(hipMemcpyAsync(out_ids, d_ids, sizeof(int32_t) * (size_t)nq * k, hipMemcpyDeviceToHost,
                          s),
           "pp outputs");
    HIPTRY(hipMemcpyAsync(out_dist, d_dist, sizeof(double) * (size_t)nq * k,
                          hipMemcpyDeviceToHost, s),
           "pp outputs");
  }
  HIPTRY(hipStreamSynchronize(s), "pp_topk");
  return PANTHER_OK;
}

int run_pp(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, int32_t D, int32_t k,
           int32_t* d_ids, double* d_dist, hipStream_t s) {
  if (c->pp_form == PANTHER_PP_FP64) {
    const int e = launch_knn_fp64(c->d_theta, c->n, D, c->d_theta, true, dq, nullptr, nq, k, d_ids,
                                  d_dist, s);
    HIPTRY((hipError_t)e, "pp fp64 knn");
    return PANTHER_OK;
  }
  return run_pp_bf16(c, lane, dq, nq, D, k, d_ids, d_dist, s, nullptr);
}

// Cross-graph Panther++: queries are vertices of qc's graph, the database
// is every vertex of dbc's graph; each side has its own paths and features.
extern "C" int panther_pp_topk_cross(panther_ctx* qc, panther_ctx* dbc, const int32_t* queries,
                                     int64_t nq, int32_t D, int32_t k, int32_t* out_ids,
                                     double* out_dist, int mem, void* stream) {
  if (!qc || !dbc) return PANTHER_EINVAL;
  panther_ctx* const c = dbc;  // errors of the call are reported on the database context
  qc->err.clear();
  dbc->err.clear();
  if (!qc->has_paths || !dbc->has_paths)
    return ctx_fail(dbc, PANTHER_ESTATE, "pp_topk_cross before sample_paths on both graphs");
  if (qc->device != dbc->device)
    return ctx_fail(dbc, PANTHER_EINVAL, "the two contexts must be on the same device");
  if (qc == dbc) return ctx_fail(dbc, PANTHER_EINVAL, "use panther_pp_topk within one graph");
  if (D < 1 || D > 256) return ctx_fail(dbc, PANTHER_EINVAL, "D must lie in [1, 256]");
  if (k < 1 || k > 256) return ctx_fail(dbc, PANTHER_EINVAL, "k must lie in [1, 256]");
  if (nq < 0) return ctx_fail(dbc, PANTHER_EINVAL, "nq must be >= 0");
  if (mem != PANTHER_MEM_HOST && mem != PANTHER_MEM_DEVICE)
    return ctx_fail(dbc, PANTHER_EINVAL, "bad mem");
  if (nq == 0) return PANTHER_OK;
  if (!queries || !out_ids || !out_dist) return ctx_fail(dbc, PANTHER_EINVAL, "null buffer");
  if (dbc->pp_form == PANTHER_PP_BF16 && D > 64)
    return ctx_fail(dbc, PANTHER_EINVAL, "the BF16 form supports D <= 64");
  if (hipSetDevice(dbc->device) != hipSuccess)
    return ctx_fail(dbc, PANTHER_EDEVICE, "hipSetDevice");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : dbc->stream;
  std::vector<int32_t> hq;
  const int32_t* dq = nullptr;
  void* owned = nullptr;
  // query ids are checked against the query graph
  int st = stage_queries(qc, queries, nq, mem, s, hq, &dq, &owned);
  struct Own {
    void* p;
    ~Own() { ctx_free(p); }
  } own{owned};
  if (st) {
    if (qc->err.size()) dbc->err = qc->err;
    return st;
  }
  TRY(order_begin(qc, s));
  TRY(order_begin(dbc, s));
  st = ensure_features(qc, D, s);
  if (st) {
    dbc->err = qc->err;
    return st;
  }
  TRY(ensure_features(dbc, D, s));
  Lane* lane = &dbc->lane0;
  int32_t* d_ids = out_ids;
  double* d_dist = out_dist;
  if (mem == PANTHER_MEM_HOST) {
    TRY(ctx_ensure(dbc, lane->b_out, (sizeof(int32_t) + sizeof(double)) * (size_t)nq * k,
                   "pp outputs"));
    d_dist = static_cast<double*>(lane->b_out.p);
    d_ids = reinterpret_cast<int32_t*>(d_dist + (size_t)nq * k);
  }
  stage_begin(dbc, 4, s);
  if (dbc->pp_form == PANTHER_PP_FP64) {
    const int e = launch_knn_fp64(dbc->d_theta, dbc->n, D, qc->d_theta, false, dq, nullptr, nq, k,
                                  d_ids, d_dist, s);
    HIPTRY((hipError_t)e, "pp fp64 cross knn");
  } else {
    TRY(prepare_bf16(dbc, D, s));
    TRY(run_pp_bf16(dbc, lane, dq, nq, D, k, d_ids, d_dist, s, qc->d_theta));
  }
  stage_end(dbc, 4, s);
  TRY(order_end(dbc, s));
  TRY(order_end(qc, s));
  if (mem == PANTHER_MEM_HOST) {
    HIPTRY(hipMemcpyAsync(out_ids, d_ids, sizeof(int32_t) * (size_t)nq * k, hipMemcpyDeviceToHost,
                          s),
           "pp outputs");
    HIPTRY(hipMemcpyAsync(out_dist, d_dist, sizeof(double) * (size_t)nq * k,
                          hipMemcpyDeviceToHost, s),
           "pp outputs");
  }
  HIPTRY(hipStreamSynchronize(s), "pp_topk_cross");
  return PANTHER_OK;
}

extern "C" int panther_pp_certified(panther_ctx* c, int64_t* queries, int64_t* recomputed) {
  if (!c) return PANTHER_EINVAL;
  if (!c->lane0.have_stats) return ctx_fail(c, PANTHER_ESTATE, "no BF16 Panther++ call");
  if (queries) *queries = c->lane0.stat_nq;
  if (recomputed) *recomputed = c->lane0.stat_fallback;
  return PANTHER_OK;
}

extern "C" int panther_pp_scanned(panther_ctx* c, double* fraction) {
  if (!c || !fraction) return PANTHER_EINVAL;
  if (!c->lane0.have_stats) return ctx_fail(c, PANTHER_ESTATE, "no BF16 Panther++ call");
  *fraction = c->lane0.stat_scanned;
  return PANTHER_OK;
}

extern "C" int panther_pp_stats(panther_ctx* c, double* max_rel_err, double* mean_pre_recall) {
  if (!c) return PANTHER_EINVAL;
  if (!c->lane0.have_stats) return ctx_fail(c, PANTHER_ESTATE, "no BF16 Panther++ call");
  if (max_rel_err) *max_rel_err = c->lane0.max_rel_err;
  if (mean_pre_recall) *mean_pre_recall = c->lane0.mean_pre_recall;
  return PANTHER_OK;
}
