/*
 * Plain CPU oracle for the Panther hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code, header,
 * table or constant with the HIP library; the two meet only through the
 * seeded synthetic inputs.
 *
 * Paper: J. Zhang, J. Tang, C. Ma, H. Tong, Y. Jing, J. Li, "Panther: Fast
 * Top-k Similarity Search in Large Networks" (KDD 2015, arXiv:1504.02577).
 *
 * Every routine is written for obviousness, not speed: no blocking, no
 * fusion, no reordering beyond what the cited passage states.  Where the
 * paper leaves a detail open, the reading taken is stated next to the code.
 *
 * Random bits: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), written from that paper's
 * definition.  For path pid and step t (t = 0 picks the start vertex):
 *     key     = (seed mod 2^32, seed >> 32)
 *     counter = (t, 0, pid mod 2^32, pid >> 32)
 *     r       = x0 | (x1 << 32)      (x2, x3 unused)
 *
 * Reading of "randomly sample a neighbour according to transition
 * probabilities" (Algorithm GenerateRandomPath with Eq. 3): with W_v the sum
 * of the weights on v's CSR row, u = floor(r * W_v / 2^64) is a uniform
 * integer in [0, W_v) (bias <= W_v / 2^64), and the chosen edge is the first
 * CSR entry e of the row whose inclusive weight prefix exceeds u.  Each edge
 * is therefore picked with probability w_e / W_v = t_ij.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC 2011): 10 rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                           */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL_A;
      k1 += PHILOX_WEYL_B;
    }
    uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
    uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)pb;
    uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)pa;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 64-bit draw for (seed, pid, step). */
uint64_t or_draw(uint64_t seed, uint64_t pid, uint32_t step) {
  uint32_t ctr[4] = {step, 0u, (uint32_t)pid, (uint32_t)(pid >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  or_philox4x32_10(ctr, key, x);
  return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
}

/* floor(r * n / 2^64): maps a uniform 64-bit word onto [0, n). */
uint64_t or_scale(uint64_t r, uint64_t n) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* ------------------------------------------------------------------------ */
/* Graph (Section 2, Definition 1; Eq. 3).                                   */
/* ------------------------------------------------------------------------ */
/* Validates the CSR: row_ptr starts at 0, never decreases, ends at m, and
 * every column id lies in [0, n). */
int or_validate(int32_t n, int64_t m, const int32_t *row_ptr,
                const int32_t *col) {
  if (n < 1 || m < 0) return OR_EINVAL;
  if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != m) return OR_EINVAL;
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return OR_EINVAL;
  for (int64_t e = 0; e < m; ++e)
    if (col[e] < 0 || col[e] >= n) return OR_EINVAL;
  return OR_OK;
}

/* Row weight sums W_v (Eq. 3's denominator). */
void or_row_weights(int32_t n, const int32_t *row_ptr, const uint32_t *w,
                    uint64_t *W) {
  for (int32_t v = 0; v < n; ++v) {
    uint64_t s = 0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) s += w[e];
    W[v] = s;
  }
}

/* Start set: vertices with W_v > 0, ascending.  Reading: the uniform start
 * of GenerateRandomPath ranges over vertices that have a T-path at all,
 * which is what the normalisation of Eq. 1 over all T-paths implies.
 * With start_all != 0 every vertex is a start (the flag form).
 * Returns the size of the set. */
int32_t or_start_set(int32_t n, const uint64_t *W, int start_all,
                     int32_t *out) {
  int32_t k = 0;
  for (int32_t v = 0; v < n; ++v)
    if (start_all || W[v] > 0) out[k++] = v;
  return k;
}

/* Neighbour choice on row v for the uniform word r (Eq. 3): the first CSR
 * entry whose inclusive weight prefix exceeds u = floor(r * W_v / 2^64).
 * pfx holds inclusive prefix sums restarted at each row.  The search is a
 * textbook upper-bound bisection over the row's prefix.  Returns the
 * chosen CSR entry, or -1 when W_v = 0. */
int64_t or_pick_edge(const int32_t *row_ptr, const uint64_t *pfx,
                     const uint64_t *W, int32_t v, uint64_t r) {
  if (W[v] == 0) return -1;
  uint64_t u = or_scale(r, W[v]);
  int64_t lo = row_ptr[v], hi = row_ptr[v + 1] - 1; /* answer in [lo, hi] */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (pfx[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

void or_row_prefix(int32_t n, const int32_t *row_ptr, const uint32_t *w,
                   uint64_t *pfx) {
  for (int32_t v = 0; v < n; ++v) {
    uint64_t s = 0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      s += w[e];
      pfx[e] = s;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* GenerateRandomPath (Algorithm 3).                                         */
/* Reading of the garbled loop bounds: exactly R paths (pid = 0..R-1), each  */
/* with T transitions and T+1 vertices (the T-path definition of Sec. 3.1).  */
/* paths is row-major int32[R][T+1].                                         */
/* ------------------------------------------------------------------------ */
int or_walk(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
            const uint32_t *w, int32_t T, int64_t R, uint64_t seed,
            int start_all, int32_t *paths) {
  if (T < 1 || R < 1) return OR_EINVAL;
  uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t *pfx = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!W || !pfx || !starts) {
    free(W); free(pfx); free(starts);
    return OR_ENOMEM;
  }
  or_row_weights(n, row_ptr, w, W);
  or_row_prefix(n, row_ptr, w, pfx);
  int32_t ns = or_start_set(n, W, start_all, starts);
  if (ns == 0) {
    free(W); free(pfx); free(starts);
    return OR_EINVAL;
  }
#pragma omp parallel for schedule(static)
  for (int64_t pid = 0; pid < R; ++pid) {
    int32_t *p = paths + pid * (int64_t)(T + 1);
    int32_t v = starts[or_scale(or_draw(seed, (uint64_t)pid, 0u), (uint64_t)ns)];
    p[0] = v;
    for (int32_t t = 1; t <= T; ++t) {
      int64_t e = or_pick_edge(row_ptr, pfx, W, v, or_draw(seed, (uint64_t)pid, (uint32_t)t));
      if (e >= 0) v = col[e]; /* W_v = 0 (start_all form only): stay */
      p[t] = v;
    }
  }
  free(W); free(pfx); free(starts);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Vertex-to-path inverted index (Sec. 3.1; Algorithm 3 "add p_r into P_v"). */
/* Reading: P_v is a set; a path that visits v several times is listed once. */
/* Lists are in ascending path id because paths are visited in id order.    */
/* ------------------------------------------------------------------------ */
static int or_first_occurrence(const int32_t *p, int32_t i) {
  for (int32_t j = 0; j < i; ++j)
    if (p[j] == p[i]) return 0;
  return 1;
}

/* Writes inv_ptr[n+1]; returns nnz. */
int64_t or_index_ptr(int32_t n, int32_t T, int64_t R, const int32_t *paths,
                     int64_t *inv_ptr) {
  memset(inv_ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t pid = 0; pid < R; ++pid) {
    const int32_t *p = paths + pid * (int64_t)(T + 1);
    for (int32_t i = 0; i <= T; ++i)
      if (or_first_occurrence(p, i)) inv_ptr[p[i] + 1] += 1;
  }
  for (int32_t v = 0; v < n; ++v) inv_ptr[v + 1] += inv_ptr[v];
  return inv_ptr[n];
}

int or_index_fill(int32_t n, int32_t T, int64_t R, const int32_t *paths,
                  const int64_t *inv_ptr, uint32_t *inv_pid) {
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!cur) return OR_ENOMEM;
  memcpy(cur, inv_ptr, sizeof(int64_t) * (size_t)n);
  for (int64_t pid = 0; pid < R; ++pid) {
    const int32_t *p = paths + pid * (int64_t)(T + 1);
    for (int32_t i = 0; i <= T; ++i)
      if (or_first_occurrence(p, i)) inv_pid[cur[p[i]]++] = (uint32_t)pid;
  }
  free(cur);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Panther query (Algorithm 1) and the top-k step.                           */
/* For q: every path p in P_q adds one to c(q, v) for each distinct v != q   */
/* on p, so c(q, v) = |P_q intersect P_v| and S_RP = c / R (Eq. 4).          */
/* Readings: q is excluded from its own result (Problem 1 asks for other     */
/* vertices); ranking uses the integer count, ties by ascending vertex id;   */
/* fewer than k candidates are padded with (-1, 0).                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t c;
  int32_t v;
} or_cand;

static int or_cand_cmp(const void *a, const void *b) {
  const or_cand *x = (const or_cand *)a, *y = (const or_cand *)b;
  if (x->c != y->c) return x->c > y->c ? -1 : 1;
  return (x->v > y->v) - (x->v < y->v);
}

/* Accumulates the counts of q into cnt (dense, zero on entry) and lists the
 * touched vertices; returns their number. */
static int64_t or_count_one(int32_t q, int32_t T, const int32_t *paths,
                            const int64_t *inv_ptr, const uint32_t *inv_pid,
                            uint32_t *cnt, int32_t *touched) {
  int64_t nt = 0;
  for (int64_t j = inv_ptr[q]; j < inv_ptr[q + 1]; ++j) {
    const int32_t *p = paths + (int64_t)inv_pid[j] * (int64_t)(T + 1);
    for (int32_t i = 0; i <= T; ++i) {
      int32_t v = p[i];
      if (v == q || !or_first_occurrence(p, i)) continue;
      if (cnt[v] == 0) touched[nt++] = v;
      cnt[v] += 1;
    }
  }
  return nt;
}

/* Dense counts of one query, for cross-checks: out[v] = c(q, v), out[q] = 0. */
int or_counts_dense(int32_t n, int32_t T, const int32_t *paths,
                    const int64_t *inv_ptr, const uint32_t *inv_pid, int32_t q,
                    uint32_t *out) {
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!touched) return OR_ENOMEM;
  memset(out, 0, sizeof(uint32_t) * (size_t)n);
  or_count_one(q, T, paths, inv_ptr, inv_pid, out, touched);
  free(touched);
  return OR_OK;
}

int or_topk(int32_t n, int32_t T, const int32_t *paths, const int64_t *inv_ptr,
            const uint32_t *inv_pid, const int32_t *queries, int64_t nq,
            int32_t k, int32_t *out_ids, uint32_t *out_counts,
            int32_t *out_len) {
  if (k < 1) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel
  {
    uint32_t *cnt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    or_cand *cand = (or_cand *)malloc(sizeof(or_cand) * (size_t)n);
    if (!cnt || !touched || !cand) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < nq; ++i) {
        int32_t q = queries[i];
        int64_t nt = or_count_one(q, T, paths, inv_ptr, inv_pid, cnt, touched);
        for (int64_t j = 0; j < nt; ++j) {
          cand[j].v = touched[j];
          cand[j].c = cnt[touched[j]];
          cnt[touched[j]] = 0;
        }
        qsort(cand, (size_t)nt, sizeof(or_cand), or_cand_cmp);
        int64_t take = nt < k ? nt : k;
        for (int32_t j = 0; j < k; ++j) {
          out_ids[i * k + j] = j < take ? cand[j].v : -1;
          out_counts[i * k + j] = j < take ? cand[j].c : 0u;
        }
        out_len[i] = (int32_t)take;
      }
    }
    free(cnt); free(touched); free(cand);
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* Panther++ (Sec. 3.3; Algorithm 2).                                        */
/* theta(v)[d] = the d-th largest S_RP(v, u) over u != v, i.e.               */
/* (float)c_(d) / (float)R in IEEE single precision, zero-padded to D.        */
/* ------------------------------------------------------------------------ */
int or_features(int32_t n, int32_t T, int64_t R, const int32_t *paths,
                const int64_t *inv_ptr, const uint32_t *inv_pid, int32_t D,
                float *theta) {
  if (D < 1) return OR_EINVAL;
  int status = OR_OK;
  const float fR = (float)R;
#pragma omp parallel
  {
    uint32_t *cnt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    or_cand *cand = (or_cand *)malloc(sizeof(or_cand) * (size_t)n);
    if (!cnt || !touched || !cand) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int64_t v = 0; v < n; ++v) {
        int64_t nt = or_count_one((int32_t)v, T, paths, inv_ptr, inv_pid, cnt, touched);
        for (int64_t j = 0; j < nt; ++j) {
          cand[j].v = touched[j];
          cand[j].c = cnt[touched[j]];
          cnt[touched[j]] = 0;
        }
        qsort(cand, (size_t)nt, sizeof(or_cand), or_cand_cmp);
        for (int32_t d = 0; d < D; ++d)
          theta[v * D + d] = d < nt ? (float)cand[d].c / fR : 0.0f;
      }
    }
    free(cnt); free(touched); free(cand);
  }
  return status;
}

/* Squared Euclidean distance in double precision, one fused multiply-add
 * per coordinate in coordinate order. */
double or_dist2(const float *a, const float *b, int32_t D) {
  double s = 0.0;
  for (int32_t d = 0; d < D; ++d) {
    double diff = (double)a[d] - (double)b[d];
    s = fma(diff, diff, s);
  }
  return s;
}

/* Exact k nearest neighbours of each query over all v != q, ordered by
 * (squared distance ascending, id ascending); out_dist holds the Euclidean
 * distance sqrt(d2).  S_{RP++} = 1 / distance is a monotone transform, so
 * ranking by distance is ranking by similarity.  The kd-tree of the paper
 * is an index over this same exact search, so brute force defines the
 * result.  Fewer than k others: padded with (-1, +inf). */
int or_knn(int32_t n, int32_t D, const float *theta, const int32_t *queries,
           int64_t nq, int32_t k, int32_t *out_ids, double *out_dist) {
  if (k < 1 || D < 1) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!bd || !bi) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < nq; ++i) {
        int32_t q = queries[i];
        const float *tq = theta + (int64_t)q * D;
        int32_t have = 0;
        for (int32_t v = 0; v < n; ++v) {
          if (v == q) continue;
          double d2 = or_dist2(tq, theta + (int64_t)v * D, D);
          /* keep the k best (d2, v) pairs in a sorted array; v increases,
           * so an equal d2 never displaces an earlier id */
          if (have == k && !(d2 < bd[k - 1])) continue;
          int32_t pos = have < k ? have : k - 1;
          while (pos > 0 && d2 < bd[pos - 1]) {
            bd[pos] = bd[pos - 1];
            bi[pos] = bi[pos - 1];
            --pos;
          }
          bd[pos] = d2;
          bi[pos] = v;
          if (have < k) ++have;
        }
        for (int32_t j = 0; j < k; ++j) {
          out_ids[i * k + j] = j < have ? bi[j] : -1;
          out_dist[i * k + j] = j < have ? sqrt(bd[j]) : INFINITY;
        }
      }
    }
    free(bd); free(bi);
  }
  return status;
}

/* Cross-graph nearest neighbours (Sec. 3.3 applied across two networks, the
 * identity-resolution setting of Fig. 1a): query i has the feature row
 * theta_q[i] of its own graph; the database is every row v of the other
 * graph's theta_db.  All nq_db rows are candidates (the query is not one of
 * them); order (squared distance ascending, id ascending); padding
 * (-1, +inf) when nq_db < k. */
int or_knn_cross(int32_t D, int64_t nq, const float *theta_q, int32_t n_db,
                 const float *theta_db, int32_t k, int32_t *out_ids, double *out_dist) {
  if (k < 1 || D < 1) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!bd || !bi) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < nq; ++i) {
        const float *tq = theta_q + i * D;
        int32_t have = 0;
        for (int32_t v = 0; v < n_db; ++v) {
          double d2 = or_dist2(tq, theta_db + (int64_t)v * D, D);
          if (have == k && !(d2 < bd[k - 1])) continue;
          int32_t pos = have < k ? have : k - 1;
          while (pos > 0 && d2 < bd[pos - 1]) {
            bd[pos] = bd[pos - 1];
            bi[pos] = bi[pos - 1];
            --pos;
          }
          bd[pos] = d2;
          bi[pos] = v;
          if (have < k) ++have;
        }
        for (int32_t j = 0; j < k; ++j) {
          out_ids[i * k + j] = j < have ? bi[j] : -1;
          out_dist[i * k + j] = j < have ? sqrt(bd[j]) : INFINITY;
        }
      }
    }
    free(bd); free(bi);
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* Sample size (Sec. 3.2): Theorem 1 with the VC bound of Lemma 1,           */
/* R = c / eps^2 * (log2 C(T,2) + 1 + ln(1/delta)), rounded up.              */
/* ------------------------------------------------------------------------ */
int64_t or_sample_size(double eps, double c, double delta, int32_t T) {
  if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0) || !(c > 0.0) || T < 2)
    return OR_EINVAL;
  double pairs = (double)T * (double)(T - 1) / 2.0;
  double r = c / (eps * eps) * (log2(pairs) + 1.0 + log(1.0 / delta));
  return (int64_t)ceil(r);
}

/* Paths of selected ids only (same draws as or_walk), for spot checks of
 * runs too large to replay whole. out is int32[npids][T+1]. */
int or_walk_pids(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                 const uint32_t *w, int32_t T, uint64_t seed, int start_all,
                 const int64_t *pids, int64_t npids, int32_t *out) {
  if (T < 1) return OR_EINVAL;
  uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t *pfx = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!W || !pfx || !starts) {
    free(W); free(pfx); free(starts);
    return OR_ENOMEM;
  }
  or_row_weights(n, row_ptr, w, W);
  or_row_prefix(n, row_ptr, w, pfx);
  int32_t ns = or_start_set(n, W, start_all, starts);
  for (int64_t i = 0; i < npids && ns > 0; ++i) {
    uint64_t pid = (uint64_t)pids[i];
    int32_t *p = out + i * (int64_t)(T + 1);
    int32_t v = starts[or_scale(or_draw(seed, pid, 0u), (uint64_t)ns)];
    p[0] = v;
    for (int32_t t = 1; t <= T; ++t) {
      int64_t e = or_pick_edge(row_ptr, pfx, W, v, or_draw(seed, pid, (uint32_t)t));
      if (e >= 0) v = col[e];
      p[t] = v;
    }
  }
  free(W); free(pfx); free(starts);
  return ns > 0 ? OR_OK : OR_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Counts of Algorithm 1 and the list lengths of the inverted index         */
/* (Sec. 3.1) computed by streaming over every sampled path, storing        */
/* neither the paths nor the index, for runs whose index is too large to    */
/* hold (more than 2^32 entries).  Path pid is drawn exactly as in or_walk. */
/*   list_len[v]      = |P_v|, the number of paths whose vertex set has v;  */
/*   counts[i * n + v] = c(queries[i], v) = |P_q intersect P_v| for v != q, */
/*                       and 0 for v == q.                                  */
/* Memory: one dense n-counter array per query (and per thread), so this   */
/* is meant for small graphs.                                               */
/* ------------------------------------------------------------------------ */
int or_stream_counts(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                     const uint32_t *w, int32_t T, int64_t R, uint64_t seed,
                     int start_all, const int32_t *queries, int32_t nq,
                     uint64_t *list_len, uint32_t *counts) {
  if (T < 1 || R < 1 || nq < 0) return OR_EINVAL;
  uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t *pfx = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!W || !pfx || !starts) {
    free(W); free(pfx); free(starts);
    return OR_ENOMEM;
  }
  or_row_weights(n, row_ptr, w, W);
  or_row_prefix(n, row_ptr, w, pfx);
  int32_t ns = or_start_set(n, W, start_all, starts);
  if (ns == 0) {
    free(W); free(pfx); free(starts);
    return OR_EINVAL;
  }
  memset(list_len, 0, sizeof(uint64_t) * (size_t)n);
  memset(counts, 0, sizeof(uint32_t) * (size_t)nq * (size_t)n);
  int status = OR_OK;
#pragma omp parallel
  {
    uint64_t *my_len = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint32_t *my_cnt = (uint32_t *)calloc((size_t)nq * (size_t)n + 1, sizeof(uint32_t));
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T + 1));
    if (!my_len || !my_cnt || !p) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(static)
      for (int64_t pid = 0; pid < R; ++pid) {
        int32_t v = starts[or_scale(or_draw(seed, (uint64_t)pid, 0u), (uint64_t)ns)];
        p[0] = v;
        for (int32_t t = 1; t <= T; ++t) {
          int64_t e = or_pick_edge(row_ptr, pfx, W, v, or_draw(seed, (uint64_t)pid, (uint32_t)t));
          if (e >= 0) v = col[e];
          p[t] = v;
        }
        /* the path's vertex set: first occurrences only */
        for (int32_t i = 0; i <= T; ++i)
          if (or_first_occurrence(p, i)) my_len[p[i]] += 1;
        for (int32_t qi = 0; qi < nq; ++qi) {
          int32_t q = queries[qi], has = 0;
          for (int32_t i = 0; i <= T; ++i) has |= p[i] == q;
          if (!has) continue;
          uint32_t *c = my_cnt + (size_t)qi * (size_t)n;
          for (int32_t i = 0; i <= T; ++i)
            if (p[i] != q && or_first_occurrence(p, i)) c[p[i]] += 1;
        }
      }
#pragma omp critical
      {
        for (int32_t v = 0; v < n; ++v) list_len[v] += my_len[v];
        for (size_t i = 0; i < (size_t)nq * (size_t)n; ++i) counts[i] += my_cnt[i];
      }
    }
    free(my_len); free(my_cnt); free(p);
  }
  free(W); free(pfx); free(starts);
  return status;
}

/* Thread count of the OpenMP loops above (timing of the CPU baseline only;
 * results do not depend on it). */
#ifdef _OPENMP
#include <omp.h>
#endif
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
