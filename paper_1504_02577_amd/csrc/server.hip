// Serving loop: continuous batching of Panther and Panther++ requests over
// resident paths, index and features.
//
// Requests enter a queue (panther_server_submit, any host thread).  A
// scheduler thread admits them, oldest first, into a batch for a free lane
// while the device memory the batch needs fits the lane's share of the
// budget (budget / lanes), and hands the batch to the lane.  A batch's need
// is computed with the same sizes the lane's kernels allocate with: for a
// Panther request, from its path-list length (a hub query's staging grows
// with T * |P_q|); for the Panther++ requests, the candidate pools of a call
// of that many queries.  A lane whose held scratch plus the next batch's
// need would exceed its share frees its scratch first, so the lanes never
// hold more than the budget between them.  Every lane has its own HIP
// stream, host worker thread and query scratch, so batches of different
// lanes run on the device at the same time while later requests keep being
// admitted.  A batch runs its Panther
// requests as one batched top-k call with k = the largest k asked (the top-k
// of a request is the prefix of that list, since the ranking is a total
// order) and its Panther++ requests as one Panther++ call likewise.
// Completed results, each with its latency from submission, are collected by
// panther_server_poll.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/panther.h"
#include "runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t tag;
  int32_t kind;
  int32_t q;
  int32_t k;
  double t_submit;
  size_t mem;  // Panther: its share of a batched call; Panther++: its outputs
};

struct Batch {
  std::vector<Request> reqs;
  size_t mem_panther = 0;  // sum over its Panther requests
  size_t mem_pp = 0;       // sum over its Panther++ requests' outputs
  int64_t n_pp = 0;
  size_t mem = 0;          // device bytes the batch needs on its lane
};

struct LaneWorker {
  Lane lane;
  hipStream_t stream = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool has_batch = false;
  Batch batch;
  bool busy = false;
  // pinned host staging
  int32_t* h_q = nullptr;
  int32_t* h_ids = nullptr;
  uint32_t* h_cnt = nullptr;
  int32_t* h_len = nullptr;
  double* h_dist = nullptr;
  // device staging
  DevBuf d_q, d_out;
};

}  // namespace

struct panther_server {
  panther_ctx* c = nullptr;
  int64_t budget = 0;
  int32_t max_batch = 0;
  int32_t D = 0;
  std::vector<LaneWorker*> lanes;
  std::thread scheduler;
  std::mutex mu;
  std::condition_variable cv;        // pending queue / lane availability
  std::deque<Request> pending;
  size_t share = 0;                  // device bytes each lane may hold
  std::vector<uint64_t> list_ptr;    // host copy of the index offsets (|P_q|)
  BatchSizing sizing{};              // the lanes' tier limits (all lanes alike)
  std::atomic<int64_t> peak_lane{0};  // most device bytes a lane held
  std::atomic<bool> stopping{false};
  std::mutex done_mu;
  std::condition_variable done_cv;
  std::deque<panther_result> done;
  std::vector<double> latencies;
  double t_first = -1.0, t_last = 0.0;
  int64_t completed = 0;
  std::atomic<int> failures{0};
};

// Device bytes of a request's query id and output rows on its lane (a
// batch's rows are as wide as its largest k, at most PANTHER_SERVER_KMAX).
constexpr size_t kRowBytes =
    sizeof(int32_t) + PANTHER_SERVER_KMAX * (sizeof(int32_t) + sizeof(double)) + sizeof(int32_t);

static size_t request_mem(const panther_server* sv, int kind, int32_t q) {
  if (kind == 1) return kRowBytes;
  const uint64_t L = sv->list_ptr[(size_t)q + 1] - sv->list_ptr[(size_t)q];
  return kRowBytes + batched_query_bytes(sv->sizing, L, PANTHER_SERVER_KMAX);
}

// Device bytes a batch needs on a lane: the batched call's fixed buffers,
// its Panther requests' shares, and the Panther++ call of n_pp queries.
static size_t batch_mem(const panther_server* sv, size_t mem_panther, size_t mem_pp,
                        int64_t n_pp) {
  return batched_fixed_bytes() + mem_panther + mem_pp +
         pp_lane_bytes(sv->c, n_pp, PANTHER_SERVER_KMAX);
}

static size_t lane_held(LaneWorker* w) {
  return lane_device_bytes(&w->lane) + (w->d_q.p ? w->d_q.cap : 0) +
         (w->d_out.p ? w->d_out.cap : 0);
}

static void finish(panther_server* sv, const Request& r, const int32_t* ids, const uint32_t* cnt,
                   const double* dist, int32_t len, int status) {
  panther_result res;
  std::memset(&res, 0, sizeof res);
  res.tag = r.tag;
  res.kind = r.kind;
  res.query = r.q;
  res.k = r.k;
  res.status = status;
  int32_t n = std::min(len, r.k);
  res.len = status == PANTHER_OK ? n : 0;
  for (int32_t j = 0; j < r.k && j < PANTHER_SERVER_KMAX; ++j) {
    const bool ok = status == PANTHER_OK && j < n;
    res.ids[j] = ok ? ids[j] : -1;
    res.scores[j] = ok ? (r.kind == 0 ? (double)cnt[j] : dist[j]) : (r.kind == 0 ? 0.0 : INFINITY);
  }
  const double t = now_ms();
  res.latency_ms = t - r.t_submit;
  std::lock_guard<std::mutex> g(sv->done_mu);
  sv->done.push_back(res);
  sv->latencies.push_back(res.latency_ms);
  if (sv->t_first < 0) sv->t_first = r.t_submit;
  sv->t_last = t;
  ++sv->completed;
  sv->done_cv.notify_all();
}

// Runs one batch on a lane (worker thread).
static void run_batch(panther_server* sv, LaneWorker* w, Batch& b) {
  panther_ctx* c = sv->c;
  hipStream_t s = w->stream;
  std::vector<const Request*> pan, ppr;
  for (const Request& r : b.reqs) (r.kind == 0 ? pan : ppr).push_back(&r);
  for (int kind = 0; kind < 2; ++kind) {
    const auto& list = kind == 0 ? pan : ppr;
    if (list.empty()) continue;
    const int64_t nq = (int64_t)list.size();
    int32_t kmax = 1;
    for (const Request* r : list) kmax = std::max(kmax, r->k);
    for (int64_t i = 0; i < nq; ++i) w->h_q[i] = list[i]->q;
    int st = ctx_ensure(c, w->d_q, sizeof(int32_t) * (size_t)nq, "server queries");
    const size_t out_bytes = (size_t)nq * kmax * (sizeof(int32_t) + sizeof(double)) +
                             sizeof(int32_t) * (size_t)nq;
    if (!st) st = ctx_ensure(c, w->d_out, out_bytes, "server outputs");
    int32_t* dq = static_cast<int32_t*>(w->d_q.p);
    char* o = static_cast<char*>(w->d_out.p);
    int32_t* d_ids = reinterpret_cast<int32_t*>(o);
    double* d_dist = reinterpret_cast<double*>(o + sizeof(int32_t) * (size_t)nq * kmax);
    uint32_t* d_cnt = reinterpret_cast<uint32_t*>(d_dist);
    int32_t* d_len = reinterpret_cast<int32_t*>(o + out_bytes - sizeof(int32_t) * (size_t)nq);
    if (!st)
      st = ctx_hip(c, hipMemcpyAsync(dq, w->h_q, sizeof(int32_t) * (size_t)nq,
                                     hipMemcpyHostToDevice, s),
                   "server upload");
    if (!st && kind == 0) {
      const uint64_t* qlen = nullptr;
      st = query_lengths(c, &w->lane, dq, nq, s, &qlen, !batched_plan_on_device(nq));
      if (!st)
        st = run_batched(c, &w->lane, dq, qlen, nq, kmax, d_ids, d_cnt, d_len, nullptr, s);
      if (!st)
        st = ctx_hip(c, hipMemcpyAsync(w->h_cnt, d_cnt, sizeof(uint32_t) * (size_t)nq * kmax,
                                       hipMemcpyDeviceToHost, s),
                     "server download");
      if (!st)
        st = ctx_hip(c, hipMemcpyAsync(w->h_len, d_len, sizeof(int32_t) * (size_t)nq,
                                       hipMemcpyDeviceToHost, s),
                     "server download");
    } else if (!st) {
      st = run_pp(c, &w->lane, dq, nq, sv->D, kmax, d_ids, d_dist, s);
      if (!st)
        st = ctx_hip(c, hipMemcpyAsync(w->h_dist, d_dist, sizeof(double) * (size_t)nq * kmax,
                                       hipMemcpyDeviceToHost, s),
                     "server download");
    }
    if (!st)
      st = ctx_hip(c, hipMemcpyAsync(w->h_ids, d_ids, sizeof(int32_t) * (size_t)nq * kmax,
                                     hipMemcpyDeviceToHost, s),
                   "server download");
    if (!st) st = ctx_hip(c, hipStreamSynchronize(s), "server batch");
    if (st) sv->failures++;
    for (int64_t i = 0; i < nq; ++i) {
      const Request& r = *list[i];
      int32_t len = 0;
      if (!st) {
        if (kind == 0) {
          len = w->h_len[i];
        } else {
          len = 0;
          while (len < kmax && w->h_ids[i * kmax + len] >= 0) ++len;
        }
      }
      finish(sv, r, w->h_ids + i * kmax, kind == 0 ? w->h_cnt + i * kmax : nullptr,
             kind == 1 ? w->h_dist + i * kmax : nullptr, len, st);
    }
  }
}

static void lane_main(panther_server* sv, LaneWorker* w) {
  (void)hipSetDevice(sv->c->device);
  while (true) {
    Batch b;
    {
      std::unique_lock<std::mutex> lk(w->mu);
      w->cv.wait(lk, [&] { return w->has_batch || sv->stopping.load(); });
      if (!w->has_batch) return;
      b = std::move(w->batch);
      w->has_batch = false;
    }
    // buffers only grow within a call: if what the lane keeps plus what this
    // batch may add could pass the lane's share, start from nothing
    if (lane_held(w) + b.mem > sv->share) {
      (void)hipStreamSynchronize(w->stream);
      free_lane(&w->lane);
      ctx_release(w->d_q);
      ctx_release(w->d_out);
    }
    run_batch(sv, w, b);
    const int64_t held = (int64_t)lane_held(w);
    for (int64_t cur = sv->peak_lane.load(); held > cur &&
                                             !sv->peak_lane.compare_exchange_weak(cur, held);) {
    }
    {
      std::lock_guard<std::mutex> g(sv->mu);
      w->busy = false;
    }
    sv->cv.notify_all();
  }
}

static void scheduler_main(panther_server* sv) {
  (void)hipSetDevice(sv->c->device);
  while (true) {
    std::unique_lock<std::mutex> lk(sv->mu);
    // wake when a request can start: a lane is free (every request fits a
    // lane's share on its own, which submit checked)
    sv->cv.wait(lk, [&] {
      if (sv->pending.empty()) return sv->stopping.load();
      bool lane_free = false;
      for (LaneWorker* w : sv->lanes) lane_free = lane_free || !w->busy;
      return lane_free;
    });
    if (sv->pending.empty() && sv->stopping.load()) return;
    LaneWorker* lane = nullptr;
    for (LaneWorker* w : sv->lanes)
      if (!w->busy) {
        lane = w;
        break;
      }
    if (!lane) continue;
    // admission: the oldest requests, in order, while the batch's device
    // memory fits the lane's share
    Batch b;
    while (!sv->pending.empty() && (int32_t)b.reqs.size() < sv->max_batch) {
      const Request& r = sv->pending.front();
      const size_t mp = b.mem_panther + (r.kind == 0 ? r.mem : 0);
      const size_t mq = b.mem_pp + (r.kind == 1 ? r.mem : 0);
      const int64_t npp = b.n_pp + (r.kind == 1 ? 1 : 0);
      const size_t need = batch_mem(sv, mp, mq, npp);
      if (need > sv->share && !b.reqs.empty()) break;
      b.mem_panther = mp;
      b.mem_pp = mq;
      b.n_pp = npp;
      b.mem = need;
      b.reqs.push_back(r);
      sv->pending.pop_front();
    }
    if (b.reqs.empty()) continue;
    lane->busy = true;
    lk.unlock();
    {
      std::lock_guard<std::mutex> g(lane->mu);
      lane->batch = std::move(b);
      lane->has_batch = true;
    }
    lane->cv.notify_one();
  }
}

extern "C" int panther_server_start(panther_ctx* c, int64_t mem_budget_bytes, int32_t max_batch,
                                    int32_t lanes, int32_t D, panther_server** out) {
  if (!c || !out) return PANTHER_EINVAL;
  *out = nullptr;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "server_start before sample_paths");
  if (mem_budget_bytes < 4096) return ctx_fail(c, PANTHER_EINVAL, "memory budget too small");
  if (max_batch < 1 || max_batch > (1 << 20)) return ctx_fail(c, PANTHER_EINVAL, "bad max_batch");
  if (lanes < 1 || lanes > 8) return ctx_fail(c, PANTHER_EINVAL, "lanes must lie in [1, 8]");
  if (D < 0 || D > 256) return ctx_fail(c, PANTHER_EINVAL, "D must lie in [0, 256]");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  if (D > 0) {
    TRY(ensure_features(c, D, c->stream));
    if (c->pp_form == PANTHER_PP_BF16) TRY(prepare_bf16(c, D, c->stream));
    HIPTRY(hipStreamSynchronize(c->stream), "server features");
  }
  panther_server* sv = new panther_server();
  sv->c = c;
  sv->budget = mem_budget_bytes;
  sv->share = (size_t)mem_budget_bytes / (size_t)lanes;
  sv->max_batch = max_batch;
  sv->D = D;
  // path-list lengths on the host, for the admission estimate of each
  // Panther request
  sv->list_ptr.resize((size_t)c->n + 1);
  int st = ctx_hip(c, hipMemcpy(sv->list_ptr.data(), c->d_inv_ptr,
                                sizeof(uint64_t) * ((size_t)c->n + 1), hipMemcpyDeviceToHost),
                   "server list offsets");
  for (int i = 0; i < lanes && !st; ++i) {
    LaneWorker* w = new LaneWorker();
    sv->lanes.push_back(w);
    copy_batch_options(c, &w->lane);
    st = ctx_hip(c, hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking), "server stream");
    const size_t kcap = (size_t)max_batch * PANTHER_SERVER_KMAX;
    if (!st) st = ctx_hip(c, hipHostMalloc((void**)&w->h_q, 4 * (size_t)max_batch), "pinned");
    if (!st) st = ctx_hip(c, hipHostMalloc((void**)&w->h_ids, 4 * kcap), "pinned");
    if (!st) st = ctx_hip(c, hipHostMalloc((void**)&w->h_cnt, 4 * kcap), "pinned");
    if (!st) st = ctx_hip(c, hipHostMalloc((void**)&w->h_len, 4 * (size_t)max_batch), "pinned");
    if (!st) st = ctx_hip(c, hipHostMalloc((void**)&w->h_dist, 8 * kcap), "pinned");
  }
  if (st) {
    for (LaneWorker* w : sv->lanes) {
      if (w->stream) (void)hipStreamDestroy(w->stream);
      for (void* p : {(void*)w->h_q, (void*)w->h_ids, (void*)w->h_cnt, (void*)w->h_len,
                      (void*)w->h_dist})
        if (p) (void)hipHostFree(p);
      delete w;
    }
    delete sv;
    return st;
  }
  sv->sizing = batched_sizing(c, &sv->lanes[0]->lane);  // all lanes share the options
  for (LaneWorker* w : sv->lanes) w->th = std::thread(lane_main, sv, w);
  sv->scheduler = std::thread(scheduler_main, sv);
  *out = sv;
  return PANTHER_OK;
}

extern "C" int panther_server_submit(panther_server* sv, int32_t kind, int32_t q, int32_t k,
                                     uint64_t tag) {
  if (!sv) return PANTHER_EINVAL;
  if (kind != 0 && kind != 1) return PANTHER_EINVAL;
  if (kind == 1 && sv->D == 0) return PANTHER_ESTATE;
  if (k < 1 || k > PANTHER_SERVER_KMAX || (kind == 1 && k > 256)) return PANTHER_EINVAL;
  if (q < 0 || q >= sv->c->n) return PANTHER_ERANGE;
  Request r{tag, kind, q, k, now_ms(), request_mem(sv, kind, q)};
  // the request must fit a lane's share on its own
  const size_t alone = batch_mem(sv, kind == 0 ? r.mem : 0, kind == 1 ? r.mem : 0, kind);
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stopping) return PANTHER_ESTATE;
    if (alone > sv->share) return PANTHER_ENOMEM;
    sv->pending.push_back(r);
  }
  sv->cv.notify_all();
  return PANTHER_OK;
}

extern "C" int panther_server_poll(panther_server* sv, panther_result* results, int32_t max,
                                   int32_t timeout_us) {
  if (!sv || !results || max < 1) return PANTHER_EINVAL;
  std::unique_lock<std::mutex> lk(sv->done_mu);
  if (sv->done.empty() && timeout_us > 0)
    sv->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us),
                         [&] { return !sv->done.empty(); });
  int32_t n = 0;
  while (n < max && !sv->done.empty()) {
    results[n++] = sv->done.front();
    sv->done.pop_front();
  }
  return n;
}

extern "C" int panther_server_stats(panther_server* sv, double* p50_ms, double* p99_ms,
                                    double* qps, int64_t* completed) {
  if (!sv) return PANTHER_EINVAL;
  std::vector<double> lat;
  double t0, t1;
  int64_t done;
  {
    std::lock_guard<std::mutex> g(sv->done_mu);
    lat = sv->latencies;
    t0 = sv->t_first;
    t1 = sv->t_last;
    done = sv->completed;
  }
  auto pct = [&](double p) {
    if (lat.empty()) return 0.0;
    const size_t i = std::min(lat.size() - 1, (size_t)(p * (double)(lat.size() - 1) + 0.5));
    std::nth_element(lat.begin(), lat.begin() + i, lat.end());
    return lat[i];
  };
  if (p50_ms) *p50_ms = pct(0.50);
  if (p99_ms) *p99_ms = pct(0.99);
  if (qps) *qps = (t1 > t0 && done > 0) ? (double)done / ((t1 - t0) * 1e-3) : 0.0;
  if (completed) *completed = done;
  return sv->failures.load() ? PANTHER_EDEVICE : PANTHER_OK;
}

extern "C" int panther_server_memory(panther_server* sv, int64_t* lane_share_bytes,
                                     int64_t* peak_lane_bytes) {
  if (!sv) return PANTHER_EINVAL;
  if (lane_share_bytes) *lane_share_bytes = (int64_t)sv->share;
  if (peak_lane_bytes) *peak_lane_bytes = sv->peak_lane.load();
  return PANTHER_OK;
}

extern "C" int panther_server_stop(panther_server* sv) {
  if (!sv) return PANTHER_EINVAL;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stopping = true;
  }
  sv->cv.notify_all();
  if (sv->scheduler.joinable()) sv->scheduler.join();
  for (LaneWorker* w : sv->lanes) {
    {
      std::lock_guard<std::mutex> g(w->mu);  // pairs with the lane's wait
    }
    w->cv.notify_all();
    if (w->th.joinable()) w->th.join();
  }
  const int fails = sv->failures.load();
  for (LaneWorker* w : sv->lanes) {
    (void)hipStreamSynchronize(w->stream);
    free_lane(&w->lane);
    ctx_release(w->d_q);
    ctx_release(w->d_out);
    (void)hipStreamDestroy(w->stream);
    for (void* p : {(void*)w->h_q, (void*)w->h_ids, (void*)w->h_cnt, (void*)w->h_len,
                    (void*)w->h_dist})
      if (p) (void)hipHostFree(p);
    delete w;
  }
  delete sv;
  return fails ? PANTHER_EDEVICE : PANTHER_OK;
}
