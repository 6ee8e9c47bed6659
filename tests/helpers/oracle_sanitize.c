/* Drives every entry point of the oracle (oracle/oracle.c) on a small
 * weighted graph with an isolated vertex and a zero-weight edge, under
 * AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
 * tests/test_sanitize.py).  Any out-of-bounds access, leak, overflow or
 * misaligned load aborts with a sanitizer report; a clean run prints "ok".
 * Results are checked only for consistency between entry points: the
 * oracle's values are pinned by the other CPU tests. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_validate(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col);
int or_walk(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
            const uint32_t *w, int32_t T, int64_t R, uint64_t seed, int start_all,
            int32_t *paths);
int64_t or_index_ptr(int32_t n, int32_t T, int64_t R, const int32_t *paths, int64_t *inv_ptr);
int or_index_fill(int32_t n, int32_t T, int64_t R, const int32_t *paths,
                  const int64_t *inv_ptr, uint32_t *inv_pid);
int or_topk(int32_t n, int32_t T, const int32_t *paths, const int64_t *inv_ptr,
            const uint32_t *inv_pid, const int32_t *queries, int64_t nq, int32_t k,
            int32_t *out_ids, uint32_t *out_counts, int32_t *out_len);
int or_features(int32_t n, int32_t T, int64_t R, const int32_t *paths, const int64_t *inv_ptr,
                const uint32_t *inv_pid, int32_t D, float *theta);
int or_knn(int32_t n, int32_t D, const float *theta, const int32_t *queries, int64_t nq,
           int32_t k, int32_t *out_ids, double *out_dist);
int or_knn_cross(int32_t D, int64_t nq, const float *theta_q, int32_t n_db,
                 const float *theta_db, int32_t k, int32_t *out_ids, double *out_dist);
int64_t or_sample_size(double eps, double c, double delta, int32_t T);
int or_walk_pids(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                 const uint32_t *w, int32_t T, uint64_t seed, int start_all,
                 const int64_t *pids, int64_t npids, int32_t *out);
int or_stream_counts(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                     const uint32_t *w, int32_t T, int64_t R, uint64_t seed, int start_all,
                     const int32_t *queries, int32_t nq, uint64_t *list_len, uint32_t *counts);

#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
      return 1;                                                  \
    }                                                            \
  } while (0)

/* Undirected edges {u, v, w}: a weighted triangle 0-1-2, a tail 2-3-4 whose
 * last edge weighs 0, a pendant 6-0, and the isolated vertex 5. */
static const int32_t kEdges[][3] = {{0, 1, 3}, {1, 2, 5}, {0, 2, 7}, {2, 3, 1}, {3, 4, 0},
                                    {0, 6, 2}};
enum { N = 7, NE = 6, M = 2 * NE };

static void build_csr(int32_t *row_ptr, int32_t *col, uint32_t *w) {
  int32_t deg[N] = {0};
  for (int e = 0; e < NE; ++e) {
    deg[kEdges[e][0]]++;
    deg[kEdges[e][1]]++;
  }
  row_ptr[0] = 0;
  for (int v = 0; v < N; ++v) row_ptr[v + 1] = row_ptr[v] + deg[v];
  int32_t fill[N];
  memcpy(fill, row_ptr, sizeof fill);
  for (int e = 0; e < NE; ++e) {
    const int32_t a = kEdges[e][0], b = kEdges[e][1], x = kEdges[e][2];
    col[fill[a]] = b;
    w[fill[a]++] = (uint32_t)x;
    col[fill[b]] = a;
    w[fill[b]++] = (uint32_t)x;
  }
}

static int run(int start_all) {
  int32_t row_ptr[N + 1], col[M];
  uint32_t w[M];
  build_csr(row_ptr, col, w);
  CHECK(or_validate(N, M, row_ptr, col) == 0);
  const int32_t T = 4, D = 3, k = 9; /* k above the candidate count pads rows */
  const int64_t R = 500;
  const uint64_t seed = 0x1234567890abcdefull;
  int32_t *paths = malloc(sizeof(int32_t) * (size_t)(R * (T + 1)));
  CHECK(paths != NULL);
  CHECK(or_walk(N, M, row_ptr, col, w, T, R, seed, start_all, paths) == 0);
  int64_t inv_ptr[N + 1];
  const int64_t nnz = or_index_ptr(N, T, R, paths, inv_ptr);
  CHECK(nnz >= R && nnz <= R * (T + 1));
  uint32_t *inv_pid = malloc(sizeof(uint32_t) * (size_t)nnz);
  CHECK(inv_pid != NULL);
  CHECK(or_index_fill(N, T, R, paths, inv_ptr, inv_pid) == 0);
  int32_t queries[N];
  for (int v = 0; v < N; ++v) queries[v] = v;
  int32_t ids[N * 9], len[N];
  uint32_t counts[N * 9];
  CHECK(or_topk(N, T, paths, inv_ptr, inv_pid, queries, N, k, ids, counts, len) == 0);
  float theta[N * 3];
  CHECK(or_features(N, T, R, paths, inv_ptr, inv_pid, D, theta) == 0);
  for (int v = 0; v < N; ++v)
    if (len[v] > 0) CHECK(fabsf(theta[v * D] - (float)counts[v * k] / (float)R) == 0.0f);
  int32_t kid[N * 4];
  double kd[N * 4];
  CHECK(or_knn(N, D, theta, queries, N, 4, kid, kd) == 0);
  int32_t cid[N * 4];
  double cd[N * 4];
  CHECK(or_knn_cross(D, N, theta, N, theta, 4, cid, cd) == 0);
  /* walk_pids on every id (and ids far past R) matches the walk's rows */
  int64_t pids[R + 2];
  for (int64_t i = 0; i < R; ++i) pids[i] = i;
  pids[R] = ((int64_t)1 << 40) + 3;
  pids[R + 1] = INT64_MAX;
  int32_t *again = malloc(sizeof(int32_t) * (size_t)((R + 2) * (T + 1)));
  CHECK(again != NULL);
  CHECK(or_walk_pids(N, M, row_ptr, col, w, T, seed, start_all, pids, R + 2, again) == 0);
  CHECK(memcmp(again, paths, sizeof(int32_t) * (size_t)(R * (T + 1))) == 0);
  /* streamed counts equal the index's list lengths and the top-1 counts */
  uint64_t list_len[N];
  uint32_t *dense = malloc(sizeof(uint32_t) * N * N);
  CHECK(dense != NULL);
  CHECK(or_stream_counts(N, M, row_ptr, col, w, T, R, seed, start_all, queries, N, list_len,
                         dense) == 0);
  for (int v = 0; v < N; ++v) {
    CHECK(list_len[v] == (uint64_t)(inv_ptr[v + 1] - inv_ptr[v]));
    if (len[v] > 0) CHECK(dense[(size_t)v * N + ids[v * k]] == counts[v * k]);
  }
  free(dense);
  free(again);
  free(inv_pid);
  free(paths);
  return 0;
}

int main(void) {
  /* rejected inputs return errors without touching memory they must not */
  int32_t bad_ptr[3] = {0, 2, 1};
  int32_t bad_col[2] = {0, 5};
  if (or_validate(2, 1, bad_ptr, bad_col) == 0) return 1;
  if (or_sample_size(0.0, 0.5, 0.1, 5) >= 0) return 1;
  if (or_sample_size(0.01, 0.5, 0.1, 5) <= 0) return 1;
  if (run(0) || run(1)) return 1;
  printf("ok\n");
  return 0;
}
