// Hub queries of the batched top-k: the split, on-chip counting pipeline
// (gather, bucket scatter, per-bucket LDS count and selection, merge).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace panther {

// Staged slots a bucket is sized for.  The count step's LDS table has
// 8,192 entries, so at most 5/8 of it fills (slots of one bucket repeat ids,
// and some are empty); 4,096 measured 1.7 ms slower per R-MAT 24 call, and
// 6,144 no faster.
constexpr int kBucketTarget = 5120;
// A hub query has at most 2^kMaxBucketBits buckets.
constexpr int kMaxBucketBits = 12;
// A bucket emits at most max(k, kEmitCap) candidates to the merge.
constexpr int kEmitCap = 256;

// One hub query of a chunk; offsets are relative to the chunk's buffers and
// ascend with the query's position in the chunk.
struct HubQuery {
  int32_t qi;       // index of the query in the batch
  uint32_t nb;      // its bucket count (1 .. 2^kMaxBucketBits)
  uint32_t tile0;   // first gather tile
  uint32_t stile0;  // first bucketing tile
  uint32_t bkt0;    // first bucket
  uint32_t th0;     // first per-tile bucket count (bucketing tile-major)
  uint64_t occ0;    // first staging slot (T slots per row of P_q)
  uint64_t cand0;   // first slot of its per-bucket winners
};

// Filled on the device from the query id: P_q = inv_pid[a, a + L).
struct HubList {
  uint64_t a;
  uint64_t L;
  int32_t q;
  int32_t pad;
};

struct HubArgs {
  const int32_t* queries;
  const uint64_t* inv_ptr;
  const uint32_t* inv_pid;
  const int32_t* paths;
  const HubQuery* hq;  // [nq]
  HubList* hx;         // [nq]
  int32_t* tile_owner;   // [n_tiles] gather tile -> query of the chunk
  int32_t* stile_owner;  // [n_stiles] bucketing tile -> query
  int32_t* bkt_owner;    // [n_bkt] bucket -> query
  uint64_t* bkt_cand0;   // [n_bkt] the owner's first winner slot
  uint32_t* redo;        // [n_bkt] buckets left to the rare count path
  uint32_t* redo_n;      // their number
  int32_t nq;
  int32_t T;
  int32_t k;
  uint32_t n_tiles;
  uint32_t n_stiles;
  uint32_t n_bkt;
  int32_t* stA;          // staging in row order
  int32_t* stB;          // staging in bucket order
  uint32_t* bkt_cnt;     // [n_bkt]
  uint64_t* bkt_start;   // [n_bkt + 1]
  uint32_t* bkt_fill;    // [n_bkt]
  uint32_t* th;          // per bucketing tile bucket counts (gather -> scatter)
  uint64_t* cand;        // per-bucket winners, grouped by query
  uint32_t* cand_n;      // [nq]
  int32_t* out_ids;
  uint32_t* out_counts;
  int32_t* out_len;
  float* theta;          // feature mode: row qi gets count / R
  float fR;
};

// Buckets of a hub query with `occ` staging slots: about kBucketTarget
// slots each, at most 2^max_bits.
uint32_t hub_buckets(uint64_t occ, int max_bits);
uint32_t hub_tiles(uint64_t L);
uint32_t hub_stiles(uint64_t L);
size_t hub_count_lds();
hipError_t enqueue_hub_chunk(const HubArgs& A, int stride, void* scan_temp, hipStream_t s);
hipError_t hub_set_attributes();

}  // namespace panther
