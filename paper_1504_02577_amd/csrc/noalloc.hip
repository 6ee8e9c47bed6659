// Allocation-free Panther top-k: the plain form's kernels (Algorithm 1 and
// the top-k step, one launch per query) run on a fixed device array instead
// of memory the library allocates, for callers that cannot allocate device
// memory (work under HIP graph capture, tight serving loops, harnesses that
// forbid it).
//
// The array is a file-scope device variable: each GPU the library runs on
// holds its own copy from module load until the process ends.  Its address
// on a device comes from hipGetSymbolAddress, taken once per device with
// that device current; host code passes only that address to kernels (the
// variable's name in host code is not a device address).
//
// Layout (n = the graph's vertex count): [0, 64) control words, then the
// dense counters cnt[n], then the touched list touched[n].  Every call
// clears the control words and counters with a kernel before its queries;
// every query's kernel leaves them zero again.  Calls that overlap on one
// GPU (two contexts, two streams, two threads) share the array and race.
#include <mutex>

#include "../../include/panther.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

using namespace panther;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr size_t kCtlBytes = 64;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this GPU's scratch (the current device must be
// c->device).
int scratch_address(panther_ctx* c, unsigned char** out) {
  std::lock_guard<std::mutex> g(g_mu);
  if (c->device < 0 || c->device >= kMaxDevices)
    return ctx_fail(c, PANTHER_EDEVICE, "device ordinal %d beyond the scratch table", c->device);
  if (!g_scratch[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return ctx_fail(c, PANTHER_EDEVICE, "scratch address: %s", hipGetErrorString(e));
    }
    g_scratch[c->device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[c->device]);
  return PANTHER_OK;
}

}  // namespace

// Largest vertex count whose counters and touched list fit the array.
constexpr size_t kMaxVertices = (kScratchBytes - kCtlBytes) / (2 * sizeof(uint32_t));

extern "C" int panther_topk_similar_noalloc(panther_ctx* c, const int32_t* queries, int64_t nq,
                                            int32_t k, int32_t* out_ids, uint32_t* out_counts,
                                            int32_t* out_len, void* stream) {
  if (!c) return PANTHER_EINVAL;
  c->err.clear();
  if (!c->has_paths) return ctx_fail(c, PANTHER_ESTATE, "topk before sample_paths");
  if (k < 1 || k > 1024) return ctx_fail(c, PANTHER_EINVAL, "k must lie in [1, 1024]");
  if (nq < 0) return ctx_fail(c, PANTHER_EINVAL, "nq must be >= 0");
  if ((size_t)c->n > kMaxVertices)
    return ctx_fail(c, PANTHER_EINVAL,
                    "the allocation-free form holds counters for at most %zu vertices "
                    "(%zu MiB of scratch); this graph has %d",
                    kMaxVertices, kScratchBytes >> 20, c->n);
  if (nq == 0) return PANTHER_OK;
  if (!queries || !out_ids || !out_counts || !out_len)
    return ctx_fail(c, PANTHER_EINVAL, "null buffer");
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, PANTHER_EDEVICE, "hipSetDevice");
  unsigned char* base = nullptr;
  TRY(scratch_address(c, &base));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  TRY(order_begin(c, s));
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + kCtlBytes);
  int32_t* touched = reinterpret_cast<int32_t*>(cnt + c->n);
  // control words and counters start at zero (the previous call, on any
  // context of this GPU, may have used another graph size)
  launch_zero_u32(ctl, kCtlBytes / sizeof(uint32_t) + (uint64_t)c->n, s);
  const TopkScratch sc{cnt, touched, ctl};
  for (int64_t i = 0; i < nq; ++i)
    launch_topk_plain(c->stride, queries + i, c->n, c->d_inv_ptr, c->d_inv_pid, c->d_paths,
                      (uint64_t)c->num_cus * 256, sc, k, out_ids + i * k, out_counts + i * k,
                      out_len + i, s);
  HIPTRY(hipGetLastError(), "topk (allocation-free)");
  TRY(order_end(c, s));
  return PANTHER_OK;
}
