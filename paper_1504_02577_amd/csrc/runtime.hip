// C ABI and host runtime of the Panther library: context, device memory,
// argument validation, and the sequencing of the kernels of each call.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/panther.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

using namespace panther;

// ---------------------------------------------------------------------------
// errors and allocation
// ---------------------------------------------------------------------------
int ctx_fail(panther_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) {
    std::lock_guard<std::mutex> g(c->err_mu);
    c->err = buf;
  }
  return code;
}

int ctx_hip(panther_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return PANTHER_OK;
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return ctx_fail(c, PANTHER_ENOMEM, "%s: out of device memory", what);
  }
  return ctx_fail(c, PANTHER_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int ctx_alloc(panther_ctx* c, void** p, size_t bytes, const char* what) {
  *p = nullptr;
  bool inject = false;
  {
    std::lock_guard<std::mutex> g(c->alloc_mu);
    if (c->fail_alloc_after == 0)
      inject = true;
    else if (c->fail_alloc_after > 0)
      --c->fail_alloc_after;
  }
  if (inject) return ctx_fail(c, PANTHER_ENOMEM, "%s: allocation failure injected", what);
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return ctx_fail(c, PANTHER_ENOMEM, "%s: cannot allocate %zu bytes", what, bytes);
  }
  return PANTHER_OK;
}

void ctx_free(void* p) {
  if (p) (void)hipFree(p);
}

int ctx_ensure(panther_ctx* c, DevBuf& b, size_t bytes, const char* what) {
  if (bytes <= b.cap && b.p) return PANTHER_OK;
  ctx_free(b.p);
  b.p = nullptr;
  b.cap = 0;
  void* p;
  const int st = ctx_alloc(c, &p, bytes, what);
  if (st) return st;
  b.p = p;
  b.cap = bytes;
  return PANTHER_OK;
}

void ctx_release(DevBuf& b) {
  ctx_free(b.p);
  b.p = nullptr;
  b.cap = 0;
}

int pinned_ensure(panther_ctx* c, PinnedBuf& b, size_t bytes, const char* what) {
  if (bytes <= b.cap && b.p) return PANTHER_OK;
  pinned_release(b);
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes < 4096 ? 4096 : bytes, hipHostMallocDefault) != hipSuccess || !p)
    return ctx_fail(c, PANTHER_ENOMEM, "out of pinned host memory (%s)", what);
  b.p = p;
  b.cap = bytes < 4096 ? 4096 : bytes;
  return PANTHER_OK;
}

void pinned_release(PinnedBuf& b) {
  if (b.p) (void)hipHostFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}


static void free_features(panther_ctx* c) {
  ctx_free(c->d_theta);
  c->d_theta = nullptr;
  c->theta_D = 0;
  free_pp_state(c);
}

// Drops the paths, index and everything derived from them.  The storage of
// the paths and index is kept for the next sample_paths call unless
// `release` is set (a new graph, or destroy).
static void free_paths(panther_ctx* c, bool release) {
  free_features(c);
  forget_batch_graph(&c->lane0);
  c->d_paths = nullptr;
  c->d_inv_ptr = nullptr;
  c->d_inv_pid = nullptr;
  c->has_paths = false;
  c->nnz = 0;
  if (release) {
    free_lane(&c->lane0);
    for (DevBuf* b : {&c->b_paths, &c->b_inv_pid, &c->b_inv_ptr, &c->b_keys0, &c->b_keys1,
                      &c->b_vtmp, &c->b_hist, &c->b_offs, &c->b_stemp, &c->b_nnz, &c->b_allv, &c->b_queries,
                      &c->b_outs})
      ctx_release(*b);
    ctx_free(c->d_cnt);
    ctx_free(c->d_touched);
    ctx_free(c->d_ctl);
    c->d_cnt = nullptr;
    c->d_touched = nullptr;
    c->d_ctl = nullptr;
  }
}

static void free_graph(panther_ctx* c) {
  free_paths(c, true);
  ctx_free(c->d_col);
  ctx_free(c->d_vrec);
  ctx_free(c->d_pfx);
  ctx_free(c->d_vstart);
  ctx_free(c->d_edge);
  ctx_free(c->d_fat);
  ctx_free(c->d_start_rec);
  c->d_edge = nullptr;
  c->d_fat = nullptr;
  c->d_start_rec = nullptr;
  c->d_col = nullptr;
  c->d_vrec = nullptr;
  c->d_pfx = nullptr;
  c->d_vstart = nullptr;
  c->has_graph = false;
}

// RAII holder for temporaries of a call
struct Temp {
  std::vector<void*> ptrs;
  ~Temp() {
    for (void* p : ptrs) ctx_free(p);
  }
  void* add(void* p) {
    ptrs.push_back(p);
    return p;
  }
};

void stage_begin(panther_ctx* c, int stage, hipStream_t s) {
  if (!c->timing) return;
  if (!c->ev[0]) {
    for (int i = 0; i < 10; ++i) (void)hipEventCreate(&c->ev[i]);
  }
  (void)hipEventRecord(c->ev[2 * stage], s);
}

void stage_end(panther_ctx* c, int stage, hipStream_t s) {
  if (!c->timing) return;
  (void)hipEventRecord(c->ev[2 * stage + 1], s);
  c->ev_used[stage] = true;
}

extern "C" int panther_stage_times(panther_ctx* c, double* out_ms) {
  if (!c || !out_ms) return PANTHER_EINVAL;
  if (!c->timing) return ctx_fail(c, PANTHER_ESTATE, "timing option is off");
  for (int i = 0; i < 5; ++i) {
    out_ms[i] = -1.0;
    if (!c->ev_used[i]) continue;
    float ms = 0.f;
    if (hipEventSynchronize(c->ev[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    out_ms[i] = ms;
  }
  return PANTHER_OK;
}

int order_begin(panther_ctx* c, hipStream_t s) {
  if (!c->order_ev) {
    HIPTRY(hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming), "order event");
  }
  if (c->order_pending) HIPTRY(hipStreamWaitEvent(s, c->order_ev, 0), "order wait");
  return PANTHER_OK;
}

int order_end(panther_ctx* c, hipStream_t s) {
  HIPTRY(hipEventRecord(c->order_ev, s), "order record");
  c->order_pending = true;
  return PANTHER_OK;
}

static hipStream_t pick_stream(panther_ctx* c, void* s) {
  return s ? static_cast<hipStream_t>(s) : c->stream;
}

// ---------------------------------------------------------------------------
// create / destroy / errors / options
// ---------------------------------------------------------------------------
extern "C" int panther_create(int device_ordinal, panther_ctx** out) {
  if (!out) return PANTHER_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_ordinal < 0 || device_ordinal >= ndev) {
    (void)hipGetLastError();
    return PANTHER_EINVAL;
  }
  if (hipSetDevice(device_ordinal) != hipSuccess) return PANTHER_EDEVICE;
  panther_ctx* c = new panther_ctx();
  c->device = device_ordinal;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return PANTHER_EDEVICE;
  }
  // the cross-stream ordering event exists from the start, so that no query
  // call (the allocation-free one included) creates driver objects
  if (hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return PANTHER_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device_ordinal) == hipSuccess) {
    c->num_cus = prop.multiProcessorCount;
    c->lds_per_block = (int)prop.sharedMemPerBlock;
  }
  *out = c;
  return PANTHER_OK;
}

extern "C" void panther_destroy(panther_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_graph(c);
  for (int i = 0; i < 10; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->order_ev) (void)hipEventDestroy(c->order_ev);
  (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" const char* panther_last_error(const panther_ctx* c) {
  return c ? c->err.c_str() : "null context";
}

extern "C" int panther_set_option(panther_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return PANTHER_EINVAL;
  std::string k(key);
  if (k == "topk.form") {
    if (value != PANTHER_FORM_PLAIN && value != PANTHER_FORM_BATCHED)
      return ctx_fail(c, PANTHER_EINVAL, "topk.form must be 0 (plain) or 1 (batched)");
    c->topk_form = (int)value;
  } else if (k == "pp.form") {
    if (value != PANTHER_PP_FP64 && value != PANTHER_PP_BF16)
      return ctx_fail(c, PANTHER_EINVAL, "pp.form must be 0 (fp64) or 1 (bf16)");
    c->pp_form = (int)value;
  } else if (k == "pp.pool") {
    if (value < 32 || value > 1024)
      return ctx_fail(c, PANTHER_EINVAL, "pp.pool must lie in [32, 1024]");
    c->pp_pool = (int)value;
  } else if (k == "pp.qw") {
    if (value != 0 && value != 16 && value != 32 && value != 64)
      return ctx_fail(c, PANTHER_EINVAL, "pp.qw must be 0 (tuned), 16, 32 or 64");
    c->pp_qw = (int)value;
  } else if (k == "autotune") {
    if (value != 0 && value != 1) return ctx_fail(c, PANTHER_EINVAL, "autotune must be 0 or 1");
    c->autotune = (int)value;
  } else if (k == "timing") {
    if (value != 0 && value != 1) return ctx_fail(c, PANTHER_EINVAL, "timing must be 0 or 1");
    c->timing = (int)value;
    for (int i = 0; i < 5; ++i) c->ev_used[i] = false;
  } else if (k == "test.pp_recompute_all") {
    if (value < 0 || value > 2)
      return ctx_fail(c, PANTHER_EINVAL, "test.pp_recompute_all must be 0, 1 or 2");
    c->pp_recompute_all = (int)value;
  } else if (k == "test.fail_alloc_after") {
    c->fail_alloc_after = value < 0 ? -1 : value;
  } else if (k == "batch.tier_a" || k == "batch.tier_b" || k == "batch.block" ||
             k == "batch.wgs_per_cu" || k == "batch.hub_bits" || k == "batch.tier_b_div" ||
             k == "batch.bucket_bias" || k == "test.hub_budget") {
    return set_batch_option(c, k, value);
  } else {
    return ctx_fail(c, PANTHER_EINVAL, "unknown option '%s'", key);
  }
  return PANTHER_OK;
}

extern "C" int64_t panther_sample_size(double eps, double cc, double delta, int32_t T) {
  if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0) || !(cc > 0.0) || T < 2)
    return PANTHER_EINVAL;
  const double pairs = 0.5 * (double)T * (double)(T - 1);
  const double r = cc / (eps * eps) * (std::log2(pairs) + 1.0 + std::log(1.0 / delta));
  return (int64_t)std::ceil(r);
}

extern "C" int panther_synchronize(panther_ctx* c) {
  if (!c) return PANTHER_EINVAL;
  return ctx_hip(c, hipStreamSynchronize(c->stream), "synchronize");
}

// ---------------------------------------------------------------------------
// load_graph (a1): validate, W_v, start set, per-row prefixes
// ---------------------------------------------------------------------------
extern "C" int panther_load_graph(panther_ctx* c, int32_t n, int64_t m, const int32_t* row_ptr,
                                  const int32_t* col, const uint32_t* w, int mem,
                                  uint32_t flags) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  if (n < 1) return ctx_fail(c, PANTHER_EINVAL, "n must be >= 1");
  if (m < 0 || m >= (int64_t(1) << 31))
    return ctx_fail(c, PANTHER_EINVAL, "m must lie in [0, 2^31)");
  if (!row_ptr || (m > 0 && (!col || !w)))
    return ctx_fail(c, PANTHER_EINVAL, "null CSR pointer");
  if (mem != PANTHER_MEM_HOST && mem != PANTHER_MEM_DEVICE)
    return ctx_fail(c, PANTHER_EINVAL, "mem must be PANTHER_MEM_HOST or PANTHER_MEM_DEVICE");
  if (flags & ~(PANTHER_START_ALL_VERTICES | PANTHER_CHECK_SYMMETRIC))
    return ctx_fail(c, PANTHER_EINVAL, "unknown flags");
  hipStream_t s = c->stream;
  int32_t ends[2];
  if (mem == PANTHER_MEM_HOST) {
    ends[0] = row_ptr[0];
    ends[1] = row_ptr[n];
  } else {
    HIPTRY(hipMemcpyAsync(&ends[0], row_ptr, 4, hipMemcpyDeviceToHost, s), "load_graph");
    HIPTRY(hipMemcpyAsync(&ends[1], row_ptr + n, 4, hipMemcpyDeviceToHost, s), "load_graph");
    HIPTRY(hipStreamSynchronize(s), "load_graph");
  }
  if (ends[0] != 0 || (int64_t)ends[1] != m)
    return ctx_fail(c, PANTHER_EINVAL, "row_ptr must start at 0 and end at m");

  free_graph(c);
  Temp tmp;
  const int32_t* d_rp = row_ptr;
  const uint32_t* d_w = w;
  int32_t* d_col = nullptr;
  void* p;
  TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)m, "graph columns"));
  d_col = static_cast<int32_t*>(p);
  c->d_col = d_col;
  if (mem == PANTHER_MEM_HOST) {
    TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)(n + 1), "row_ptr staging"));
    tmp.add(p);
    HIPTRY(hipMemcpyAsync(p, row_ptr, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s),
           "row_ptr upload");
    d_rp = static_cast<const int32_t*>(p);
    TRY(ctx_alloc(c, &p, sizeof(uint32_t) * (size_t)m, "weight staging"));
    tmp.add(p);
    if (m)
      HIPTRY(hipMemcpyAsync(p, w, sizeof(uint32_t) * (size_t)m, hipMemcpyHostToDevice, s),
             "weight upload");
    d_w = static_cast<const uint32_t*>(p);
    if (m)
      HIPTRY(hipMemcpyAsync(d_col, col, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s),
             "column upload");
  } else if (m) {
    HIPTRY(hipMemcpyAsync(d_col, col, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s),
           "column copy");
  }
  // small control block: [0] error bits, [1] n_big, [2..3] max W (u64)
  TRY(ctx_alloc(c, &p, 64, "control"));
  tmp.add(p);
  uint32_t* ctl = static_cast<uint32_t*>(p);
  HIPTRY(hipMemsetAsync(ctl, 0, 64, s), "control clear");
  launch_validate(d_rp, d_col, n, m, ctl, s);
  HIPTRY(hipGetLastError(), "validate");
  uint32_t hctl[4];
  HIPTRY(hipMemcpyAsync(hctl, ctl, 16, hipMemcpyDeviceToHost, s), "validate");
  HIPTRY(hipStreamSynchronize(s), "validate");
  if (hctl[0] & 1u) {
    free_graph(c);
    return ctx_fail(c, PANTHER_EINVAL, "row_ptr decreases");
  }
  if (hctl[0] & 2u) {
    free_graph(c);
    return ctx_fail(c, PANTHER_EINVAL, "column id out of range");
  }
  if (flags & PANTHER_CHECK_SYMMETRIC) {
    TRY(ctx_alloc(c, &p, (size_t)n, "row order flags"));
    tmp.add(p);
    launch_check_symmetric(d_rp, d_col, d_w, n, static_cast<uint8_t*>(p), ctl, s);
    HIPTRY(hipGetLastError(), "symmetry check");
    HIPTRY(hipMemcpyAsync(hctl, ctl, 16, hipMemcpyDeviceToHost, s), "symmetry check");
    HIPTRY(hipStreamSynchronize(s), "symmetry check");
    if (hctl[0] & 4u) {
      free_graph(c);
      return ctx_fail(c, PANTHER_EINVAL,
                      "CSR is not symmetric: an entry v->u of weight w lacks a matching u->v "
                      "of weight w");
    }
  }
  TRY(ctx_alloc(c, &p, sizeof(VRec) * (size_t)n, "vertex records"));
  c->d_vrec = static_cast<VRec*>(p);
  TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)n, "long-row list"));
  tmp.add(p);
  int32_t* big = static_cast<int32_t*>(p);
  launch_rowsum(d_rp, d_w, n, c->d_vrec, reinterpret_cast<uint64_t*>(ctl + 2), big, ctl + 1, s);
  HIPTRY(hipGetLastError(), "rowsum");
  HIPTRY(hipMemcpyAsync(hctl, ctl, 16, hipMemcpyDeviceToHost, s), "rowsum");
  HIPTRY(hipStreamSynchronize(s), "rowsum");
  const uint32_t n_big = hctl[1];
  launch_rowsum_big(big, n_big, d_w, c->d_vrec, reinterpret_cast<uint64_t*>(ctl + 2), s);
  HIPTRY(hipGetLastError(), "rowsum_big");
  HIPTRY(hipMemcpyAsync(hctl, ctl, 16, hipMemcpyDeviceToHost, s), "rowsum");
  HIPTRY(hipStreamSynchronize(s), "rowsum");
  const uint64_t max_w = (uint64_t)hctl[2] | ((uint64_t)hctl[3] << 32);
  if (max_w >= (uint64_t(1) << 63)) {
    free_graph(c);
    return ctx_fail(c, PANTHER_EINVAL, "row weight sum exceeds 2^63");
  }
  // start set
  const int start_all = (flags & PANTHER_START_ALL_VERTICES) ? 1 : 0;
  TRY(ctx_alloc(c, &p, sizeof(uint32_t) * (size_t)n, "start flags"));
  tmp.add(p);
  uint32_t* sflags = static_cast<uint32_t*>(p);
  TRY(ctx_alloc(c, &p, sizeof(uint64_t) * (size_t)(n + 1), "start positions"));
  tmp.add(p);
  uint64_t* spos = static_cast<uint64_t*>(p);
  TRY(ctx_alloc(c, &p, scan_temp_bytes(n), "scan temp"));
  tmp.add(p);
  void* stemp = p;
  launch_start_flags(c->d_vrec, n, start_all, sflags, s);
  launch_scan_u32_to_u64(sflags, spos, n, stemp, s);
  HIPTRY(hipGetLastError(), "start set");
  uint64_t nstart = 0;
  HIPTRY(hipMemcpyAsync(&nstart, spos + n, 8, hipMemcpyDeviceToHost, s), "start set");
  HIPTRY(hipStreamSynchronize(s), "start set");
  if (nstart == 0) {
    free_graph(c);
    return ctx_fail(c, PANTHER_EINVAL, "no vertex has an edge of positive weight");
  }
  TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)nstart, "start set"));
  c->d_vstart = static_cast<int32_t*>(p);
  launch_start_scatter(sflags, spos, n, c->d_vstart, s);
  // prefixes
  c->pfx64 = max_w >= (uint64_t(1) << 32);
  TRY(ctx_alloc(c, &p, (c->pfx64 ? 8 : 4) * (size_t)m, "weight prefixes"));
  c->d_pfx = p;
  if (c->pfx64) {
    launch_prefix64(c->d_vrec, d_w, n, big, n_big, static_cast<uint64_t*>(c->d_pfx), s);
  } else {
    launch_prefix32(c->d_vrec, d_w, n, big, n_big, static_cast<uint32_t*>(c->d_pfx), s);
    TRY(ctx_alloc(c, &p, sizeof(uint2) * (size_t)m, "packed edges"));
    c->d_edge = static_cast<uint2*>(p);
    TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)m, "guide table"));
    tmp.add(p);
    int32_t* guide = static_cast<int32_t*>(p);
    TRY(ctx_alloc(c, &p, 4 * sizeof(uint4) * (size_t)m, "guide records"));
    c->d_fat = static_cast<uint4*>(p);
    launch_pack_edges(static_cast<const uint32_t*>(c->d_pfx), d_col, m, c->d_edge, s);
    launch_guide(c->d_vrec, static_cast<const uint32_t*>(c->d_pfx), n, big, n_big, guide, s);
    launch_fat_guide(c->d_vrec, static_cast<const uint32_t*>(c->d_pfx), d_col, guide, n, big,
                     n_big, c->d_fat, s);
    TRY(ctx_alloc(c, &p, sizeof(int4) * (size_t)nstart, "start records"));
    c->d_start_rec = static_cast<int4*>(p);
    launch_start_records(c->d_vstart, (int32_t)nstart, c->d_vrec, c->d_start_rec, s);
  }
  HIPTRY(hipGetLastError(), "prefix");
  HIPTRY(hipStreamSynchronize(s), "load_graph");
  c->n = n;
  c->m = m;
  c->nstart = (int32_t)nstart;
  c->max_w = max_w;
  c->has_graph = true;
  return PANTHER_OK;
}

// ---------------------------------------------------------------------------
// sample_paths (a2 walk + a3 index)
// ---------------------------------------------------------------------------
static int build_index(panther_ctx* c) {
  hipStream_t s = c->stream;
  const int32_t n = c->n;
  const uint64_t R = (uint64_t)c->R;
  int bits_total = 1;
  while (bits_total < 31 && (int64_t(1) << bits_total) < (int64_t)n) ++bits_total;
  const int passes = (bits_total + kRadixPassBits - 1) / kRadixPassBits;
  const int pass_bits = (bits_total + passes - 1) / passes;
  const uint64_t tiles1 = radix_tiles_paths(R, c->T);
  // buffers are sized for the pair count's bound R (T+1), so the passes
  // never wait for the host to learn the count
  const uint64_t nnz_cap = R * (uint64_t)(c->T + 1);
  const uint64_t tiles = radix_tiles_pairs(nnz_cap);
  const uint64_t hist_cap = 256 * std::max<uint64_t>(tiles1, tiles);
  TRY(ctx_ensure(c, c->b_hist, sizeof(uint32_t) * hist_cap, "radix histograms"));
  TRY(ctx_ensure(c, c->b_offs, sizeof(uint64_t) * (hist_cap + 1), "radix offsets"));
  TRY(ctx_ensure(c, c->b_stemp, scan_temp_bytes((int64_t)hist_cap), "scan temp"));
  TRY(ctx_ensure(c, c->b_nnz, 64, "pair count"));
  TRY(ctx_ensure(c, c->b_inv_pid, sizeof(uint32_t) * nnz_cap, "index path ids"));
  TRY(ctx_ensure(c, c->b_inv_ptr, sizeof(uint64_t) * (size_t)(n + 1), "index offsets"));
  TRY(ctx_ensure(c, c->b_keys0, sizeof(uint32_t) * nnz_cap, "radix keys"));
  if (passes > 1) TRY(ctx_ensure(c, c->b_keys1, sizeof(uint32_t) * nnz_cap, "radix keys"));
  if (passes > 1) TRY(ctx_ensure(c, c->b_vtmp, sizeof(uint32_t) * nnz_cap, "radix values"));
  uint32_t* hist = static_cast<uint32_t*>(c->b_hist.p);
  uint64_t* offs = static_cast<uint64_t*>(c->b_offs.p);
  uint64_t* d_nnz = static_cast<uint64_t*>(c->b_nnz.p);
  void* stemp = c->b_stemp.p;
  c->d_inv_pid = static_cast<uint32_t*>(c->b_inv_pid.p);
  c->d_inv_ptr = static_cast<uint64_t*>(c->b_inv_ptr.p);
  uint32_t* keys[2] = {static_cast<uint32_t*>(c->b_keys0.p),
                       static_cast<uint32_t*>(c->b_keys1.p)};
  uint32_t* vtmp = static_cast<uint32_t*>(c->b_vtmp.p);
  // pass p writes its values to inv_pid when (passes - p) is even, so the
  // last pass lands in inv_pid
  auto vals_of = [&](int pass) { return ((passes - pass) % 2 == 0) ? c->d_inv_pid : vtmp; };
  // pass 1: histograms straight from the path rows; the scan's total is
  // the pair count
  int shift = 0;
  int bits = std::min(pass_bits, bits_total - shift);
  launch_radix_up_paths(c->stride, c->d_paths, R, c->T, shift, bits, hist, s);
  launch_scan_u32_to_u64(hist, offs, (int64_t)(256 * tiles1), stemp, s);
  launch_copy_u64(offs + 256 * tiles1, d_nnz, s);
  launch_radix_down_paths(c->stride, c->d_paths, R, c->T, shift, bits, offs, keys[0], vals_of(1),
                          s);
  HIPTRY(hipGetLastError(), "index pass 1");
  for (int pass = 2; pass <= passes; ++pass) {
    shift += bits;
    bits = std::min(pass_bits, bits_total - shift);
    const uint32_t* kin = keys[(pass - 2) % 2];
    uint32_t* kout = keys[(pass - 1) % 2];
    launch_radix_up_pairs(kin, d_nnz, nnz_cap, shift, bits, hist, s);
    launch_scan_u32_to_u64(hist, offs, (int64_t)(256 * tiles), stemp, s);
    launch_radix_down_pairs(kin, vals_of(pass - 1), d_nnz, nnz_cap, shift, bits, offs, kout,
                            vals_of(pass), s);
    HIPTRY(hipGetLastError(), "index pass");
  }
  launch_list_bounds(keys[(passes - 1) % 2], d_nnz, nnz_cap, n, c->d_inv_ptr, s);
  HIPTRY(hipGetLastError(), "index bounds");
  return PANTHER_OK;
}

extern "C" int panther_sample_paths(panther_ctx* c, int32_t T, int64_t R, uint64_t seed) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_graph) return ctx_fail(c, PANTHER_ESTATE, "sample_paths before load_graph");
  if (T < 1 || T > 63) return ctx_fail(c, PANTHER_EINVAL, "T must lie in [1, 63]");
  if (R < 1 || R >= (int64_t(1) << 32)) return ctx_fail(c, PANTHER_EINVAL, "R must lie in [1, 2^32)");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  free_paths(c, false);
  int stride = 4;
  while (stride < T + 1) stride <<= 1;
  c->T = T;
  c->R = R;
  c->seed = seed;
  c->stride = stride;
  void* p;
  int st = ctx_ensure(c, c->b_paths, sizeof(int32_t) * (size_t)R * (size_t)stride, "paths");
  if (st) return st;
  c->d_paths = static_cast<int32_t*>(c->b_paths.p);
  stage_begin(c, 0, c->stream);
  if (c->pfx64)
    launch_walk64(stride, c->d_vrec, static_cast<const uint64_t*>(c->d_pfx), c->d_col,
                  c->d_vstart, c->nstart, T, (uint64_t)R, seed, c->d_paths, c->stream);
  else
    launch_walk32(stride, c->d_vrec, c->d_edge, c->d_fat, c->d_start_rec, c->nstart, T,
                  (uint64_t)R, seed, c->d_paths, c->stream);
  stage_end(c, 0, c->stream);
  st = ctx_hip(c, hipGetLastError(), "walk");
  if (!st) {
    stage_begin(c, 1, c->stream);
    st = build_index(c);
    stage_end(c, 1, c->stream);
  }
  if (!st) {
    uint64_t nnz = 0;
    st = ctx_hip(c, hipMemcpyAsync(&nnz, c->b_nnz.p, 8, hipMemcpyDeviceToHost, c->stream),
                 "pair count");
    if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "pair count");
    c->nnz = (int64_t)nnz;
  }
  if (!st && !c->d_cnt) {
    // dense per-vertex scratch of the query kernels
    st = ctx_alloc(c, &p, sizeof(uint32_t) * (size_t)c->n, "query counters");
    if (!st) {
      c->d_cnt = static_cast<uint32_t*>(p);
      st = ctx_alloc(c, &p, sizeof(int32_t) * (size_t)c->n, "query touched list");
    }
    if (!st) {
      c->d_touched = static_cast<int32_t*>(p);
      st = ctx_alloc(c, &p, 64, "query control");
    }
    if (!st) {
      c->d_ctl = static_cast<uint32_t*>(p);
      st = ctx_hip(c, hipMemsetAsync(c->d_cnt, 0, sizeof(uint32_t) * (size_t)c->n, c->stream),
                   "query scratch");
    }
    if (!st) st = ctx_hip(c, hipMemsetAsync(c->d_ctl, 0, 64, c->stream), "query scratch");
  }
  if (!st) st = ctx_hip(c, hipStreamSynchronize(c->stream), "sample_paths");
  if (st) {
    free_paths(c, true);
    return st;
  }
  c->has_paths = true;
  return PANTHER_OK;
}

// ---------------------------------------------------------------------------
// accessors
// ---------------------------------------------------------------------------
extern "C" int panther_get_paths(panther_ctx* c, int32_t* out, int mem) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "no paths sampled");
  if (!out) return ctx_fail(c, PANTHER_EINVAL, "null output");
  const size_t w = sizeof(int32_t) * (size_t)(c->T + 1);
  const size_t pitch = sizeof(int32_t) * (size_t)c->stride;
  if (mem == PANTHER_MEM_DEVICE) {
    HIPTRY(hipMemcpy2DAsync(out, w, c->d_paths, pitch, w, (size_t)c->R, hipMemcpyDeviceToDevice,
                            c->stream),
           "get_paths");
  } else {
    // rows are packed on the device chunk by chunk (a strided copy straight
    // to host memory moves one short row at a time), then copied whole
    const size_t chunk = (size_t)1 << 22;  // rows per chunk
    void* p;
    TRY(ctx_alloc(c, &p, w * std::min<size_t>(chunk, (size_t)c->R), "path staging"));
    Temp tmp;
    tmp.add(p);
    for (size_t r0 = 0; r0 < (size_t)c->R; r0 += chunk) {
      const size_t rows = std::min<size_t>(chunk, (size_t)c->R - r0);
      HIPTRY(hipMemcpy2DAsync(p, w, c->d_paths + r0 * (size_t)c->stride, pitch, w, rows,
                              hipMemcpyDeviceToDevice, c->stream),
             "get_paths");
      HIPTRY(hipMemcpyAsync(reinterpret_cast<char*>(out) + r0 * w, p, w * rows,
                            hipMemcpyDeviceToHost, c->stream),
             "get_paths");
    }
    HIPTRY(hipStreamSynchronize(c->stream), "get_paths");
    return PANTHER_OK;
  }
  HIPTRY(hipStreamSynchronize(c->stream), "get_paths");
  return PANTHER_OK;
}

extern "C" int64_t panther_index_nnz(const panther_ctx* c) {
  if (!c) return PANTHER_EINVAL;
  if (!c->has_paths) return PANTHER_ESTATE;
  return c->nnz;
}

extern "C" int panther_get_index(panther_ctx* c, int64_t* inv_ptr, uint32_t* inv_pid, int mem) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "no paths sampled");
  if (!inv_ptr || (c->nnz && !inv_pid)) return ctx_fail(c, PANTHER_EINVAL, "null output");
  const hipMemcpyKind kind =
      mem == PANTHER_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPTRY(hipMemcpyAsync(inv_ptr, c->d_inv_ptr, sizeof(int64_t) * (size_t)(c->n + 1), kind,
                        c->stream),
         "get_index");
  if (c->nnz)
    HIPTRY(hipMemcpyAsync(inv_pid, c->d_inv_pid, sizeof(uint32_t) * (size_t)c->nnz, kind,
                          c->stream),
           "get_index");
  HIPTRY(hipStreamSynchronize(c->stream), "get_index");
  return PANTHER_OK;
}

// ---------------------------------------------------------------------------
// query validation shared by topk_similar and pp_topk: returns the queries
// on the host (for range checks and the plain form's launch sizes) and on
// the device.
// ---------------------------------------------------------------------------
int stage_queries(panther_ctx* c, const int32_t* queries, int64_t nq, int mem, hipStream_t s,
                  std::vector<int32_t>& hq, const int32_t** dq, void** dq_owned) {
  *dq_owned = nullptr;
  hq.resize((size_t)nq);
  if (mem == PANTHER_MEM_HOST) {
    std::memcpy(hq.data(), queries, sizeof(int32_t) * (size_t)nq);
  } else {
    HIPTRY(hipMemcpyAsync(hq.data(), queries, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost,
                          s),
           "queries");
    HIPTRY(hipStreamSynchronize(s), "queries");
  }
  for (int64_t i = 0; i < nq; ++i)
    if (hq[i] < 0 || hq[i] >= c->n)
      return ctx_fail(c, PANTHER_ERANGE, "query %lld (= %d) outside [0, %d)", (long long)i, hq[i],
                      c->n);
  if (mem == PANTHER_MEM_DEVICE) {
    *dq = queries;
  } else {
    void* p;
    TRY(ctx_alloc(c, &p, sizeof(int32_t) * (size_t)nq, "queries"));
    *dq_owned = p;
    HIPTRY(hipMemcpyAsync(p, hq.data(), sizeof(int32_t) * (size_t)nq, hipMemcpyHostToDevice, s),
           "queries");
    *dq = static_cast<const int32_t*>(p);
  }
  return PANTHER_OK;
}

void free_lane(Lane* lane) {
  free_batch_state(lane);
  for (DevBuf* b : {&lane->b_qlen, &lane->b_pool, &lane->b_out, &lane->b_stats, &lane->b_q,
                    &lane->b_qrows, &lane->b_fb, &lane->b_fbw, &lane->b_qsort,
                    &lane->b_qsort_tmp})
    ctx_release(*b);
  pinned_release(lane->h_qlen);
  lane->have_stats = false;
}

int query_lengths(panther_ctx* c, Lane* lane, const int32_t* dq, int64_t nq, hipStream_t s,
                  const uint64_t** len, bool to_host) {
  const size_t bytes = sizeof(uint64_t) * (size_t)std::max<int64_t>(nq, 1);
  TRY(ctx_ensure(c, lane->b_qlen, bytes, "query lengths"));
  launch_query_lengths(c->d_inv_ptr, dq, nq, static_cast<uint64_t*>(lane->b_qlen.p), s);
  HIPTRY(hipGetLastError(), "query lengths");
  if (!to_host) {
    *len = nullptr;
    return PANTHER_OK;
  }
  TRY(pinned_ensure(c, lane->h_qlen, bytes, "query lengths"));
  HIPTRY(hipMemcpyAsync(lane->h_qlen.p, lane->b_qlen.p, sizeof(uint64_t) * (size_t)nq,
                        hipMemcpyDeviceToHost, s),
         "query lengths");
  HIPTRY(hipStreamSynchronize(s), "query lengths");
  *len = static_cast<const uint64_t*>(lane->h_qlen.p);
  return PANTHER_OK;
}

// ---------------------------------------------------------------------------
// all-vertex top-k: the batched form over queries 0..n-1
// ---------------------------------------------------------------------------
extern "C" int panther_topk_all(panther_ctx* c, int32_t k, int32_t* out_ids, uint32_t* out_counts,
                                int32_t* out_len, int mem, void* stream) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "topk_all before sample_paths");
  if (k < 1 || k > 1024) return ctx_fail(c, PANTHER_EINVAL, "k must lie in [1, 1024]");
  if (mem != PANTHER_MEM_HOST && mem != PANTHER_MEM_DEVICE)
    return ctx_fail(c, PANTHER_EINVAL, "bad mem");
  if (!out_ids || !out_counts || !out_len) return ctx_fail(c, PANTHER_EINVAL, "null buffer");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  hipStream_t s = pick_stream(c, stream);
  const int64_t n = c->n;
  TRY(ctx_ensure(c, c->b_allv, sizeof(int32_t) * (size_t)n, "vertex ids"));
  int32_t* ids = static_cast<int32_t*>(c->b_allv.p);
  int32_t* d_ids = out_ids;
  uint32_t* d_cnt = out_counts;
  int32_t* d_len = out_len;
  Temp tmp;
  if (mem == PANTHER_MEM_HOST) {
    void* p;
    TRY(ctx_alloc(c, &p, (sizeof(int32_t) + sizeof(uint32_t)) * (size_t)n * (size_t)k +
                             sizeof(int32_t) * (size_t)n,
                  "all-vertex outputs"));
    tmp.add(p);
    d_ids = static_cast<int32_t*>(p);
    d_cnt = reinterpret_cast<uint32_t*>(d_ids + (size_t)n * k);
    d_len = reinterpret_cast<int32_t*>(d_cnt + (size_t)n * k);
  }
  TRY(order_begin(c, s));
  stage_begin(c, 2, s);
  launch_iota(ids, (int32_t)n, s);
  HIPTRY(hipGetLastError(), "vertex ids");
  const uint64_t* qlen = nullptr;
  TRY(query_lengths(c, &c->lane0, ids, n, s, &qlen, !batched_plan_on_device(n)));
  TRY(run_batched(c, &c->lane0, ids, qlen, n, k, d_ids, d_cnt, d_len, nullptr, s));
  stage_end(c, 2, s);
  TRY(order_end(c, s));
  if (mem == PANTHER_MEM_HOST) {
    HIPTRY(hipMemcpyAsync(out_ids, d_ids, sizeof(int32_t) * (size_t)n * k, hipMemcpyDeviceToHost,
                          s),
           "all-vertex outputs");
    HIPTRY(hipMemcpyAsync(out_counts, d_cnt, sizeof(uint32_t) * (size_t)n * k,
                          hipMemcpyDeviceToHost, s),
           "all-vertex outputs");
    HIPTRY(hipMemcpyAsync(out_len, d_len, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s),
           "all-vertex outputs");
    HIPTRY(hipStreamSynchronize(s), "topk_all");
  }
  return PANTHER_OK;
}

// ---------------------------------------------------------------------------
// topk_similar (a4 + a5; a8 in the batched form)
// ---------------------------------------------------------------------------
extern "C" int panther_topk_similar(panther_ctx* c, const int32_t* queries, int64_t nq, int32_t k,
                                    int32_t* out_ids, uint32_t* out_counts, int32_t* out_len,
                                    int mem, void* stream) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "topk_similar before sample_paths");
  if (k < 1 || k > 1024) return ctx_fail(c, PANTHER_EINVAL, "k must lie in [1, 1024]");
  if (nq < 0) return ctx_fail(c, PANTHER_EINVAL, "nq must be >= 0");
  if (mem != PANTHER_MEM_HOST && mem != PANTHER_MEM_DEVICE)
    return ctx_fail(c, PANTHER_EINVAL, "bad mem");
  if (nq == 0) return PANTHER_OK;
  if (!queries || !out_ids || !out_counts || !out_len)
    return ctx_fail(c, PANTHER_EINVAL, "null buffer");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  hipStream_t s = pick_stream(c, stream);
  std::vector<int32_t> hq;
  const int32_t* dq = nullptr;
  void* owned = nullptr;
  Temp tmp;
  int st = stage_queries(c, queries, nq, mem, s, hq, &dq, &owned);
  if (owned) tmp.add(owned);
  if (st) return st;
  int32_t* d_ids = out_ids;
  uint32_t* d_cnt = out_counts;
  int32_t* d_len = out_len;
  if (mem == PANTHER_MEM_HOST) {
    void* p;
    TRY(ctx_alloc(c, &p, (sizeof(int32_t) + sizeof(uint32_t)) * (size_t)nq * (size_t)k +
                             sizeof(int32_t) * (size_t)nq,
                  "query outputs"));
    tmp.add(p);
    d_ids = static_cast<int32_t*>(p);
    d_cnt = reinterpret_cast<uint32_t*>(d_ids + (size_t)nq * k);
    d_len = reinterpret_cast<int32_t*>(d_cnt + (size_t)nq * k);
  }
  TRY(order_begin(c, s));
  stage_begin(c, 2, s);
  const uint64_t* qlen = nullptr;
  TRY(query_lengths(c, &c->lane0, dq, nq, s, &qlen,
                    c->topk_form == PANTHER_FORM_PLAIN || !batched_plan_on_device(nq)));
  if (c->topk_form == PANTHER_FORM_PLAIN) {
    TopkScratch sc{c->d_cnt, c->d_touched, c->d_ctl};
    for (int64_t i = 0; i < nq; ++i) {
      launch_topk_plain(c->stride, dq + i, c->n, c->d_inv_ptr, c->d_inv_pid, c->d_paths, qlen[i],
                        sc, k, d_ids + i * k, d_cnt + i * k, d_len + i, s);
    }
    HIPTRY(hipGetLastError(), "topk plain");
  } else {
    TRY(run_batched(c, &c->lane0, dq, qlen, nq, k, d_ids, d_cnt, d_len, nullptr, s));
  }
  stage_end(c, 2, s);
  TRY(order_end(c, s));
  if (mem == PANTHER_MEM_HOST) {
    HIPTRY(hipMemcpyAsync(out_ids, d_ids, sizeof(int32_t) * (size_t)nq * k, hipMemcpyDeviceToHost,
                          s),
           "topk outputs");
    HIPTRY(hipMemcpyAsync(out_counts, d_cnt, sizeof(uint32_t) * (size_t)nq * k,
                          hipMemcpyDeviceToHost, s),
           "topk outputs");
    HIPTRY(hipMemcpyAsync(out_len, d_len, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost, s),
           "topk outputs");
    HIPTRY(hipStreamSynchronize(s), "topk");
  } else if (owned) {
    // the staged query copy is freed on return; make sure it is consumed
    HIPTRY(hipStreamSynchronize(s), "topk");
  }
  return PANTHER_OK;
}
