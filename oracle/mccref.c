/*
 * mccref: plain sequential CPU oracle for median consensus clustering.
 *
 * TEST INFRASTRUCTURE ONLY (see mccref.h).  Written for clarity, not speed:
 * every count is recomputed from scratch by sorting, every objective value
 * by its definition as a sum of Mirkin distances.
 *
 * Notation follows the paper: k input partitions P_1..P_k, consensus C,
 * co-clustering distance delta_uv = number of partitions splitting u and v.
 */
#include "mccref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small helpers                                                              */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Sort keys[0..n) and return the sum over distinct values of count^2. */
static int64_t sum_sq_counts(int64_t* keys, int64_t n) {
  qsort(keys, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t total = 0, run = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j > 0 && keys[j] != keys[j - 1]) {
      total += run * run;
      run = 0;
    }
    ++run;
  }
  total += run * run;
  return total;
}

static int64_t pair_key(int32_t a, int32_t b) {
  return ((int64_t)a << 32) | (int64_t)(uint32_t)b;
}

/* Number of occurrences of `key` in the sorted array s[0..n). */
static int64_t count_in_sorted(const int64_t* s, int64_t n, int64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) { /* first index with s[i] >= key */
    int64_t mid = lo + (hi - lo) / 2;
    if (s[mid] < key) lo = mid + 1; else hi = mid;
  }
  int64_t first = lo;
  hi = n;
  while (lo < hi) { /* first index with s[i] > key */
    int64_t mid = lo + (hi - lo) / 2;
    if (s[mid] <= key) lo = mid + 1; else hi = mid;
  }
  return lo - first;
}

static int labels_ok(const int32_t* labels, int64_t count) {
  for (int64_t j = 0; j < count; ++j)
    if (labels[j] < 0) return 0;
  return 1;
}

static int csr_ok(const int64_t* row_ptr, const int32_t* col, int64_t n) {
  if (row_ptr[0] != 0) return 0;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return 0;
  for (int64_t j = 0; j < row_ptr[n]; ++j)
    if (col[j] < 0 || col[j] >= n) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Mirkin distance and the objective                                         */
/* ------------------------------------------------------------------------ */
/* Mirkin(A, B) = sum_a |A_a|^2 + sum_b |B_b|^2 - 2 sum_{a,b} |A_a n B_b|^2:
 * the ordered pairs co-clustered in exactly one of A and B (Appendix,
 * Eq. distance, written with cluster sizes instead of pair indicators). */
static int64_t mirkin_plain(const int32_t* a, const int32_t* b, int64_t n, int64_t* buf) {
  for (int64_t j = 0; j < n; ++j) buf[j] = a[j];
  int64_t sa = sum_sq_counts(buf, n);
  for (int64_t j = 0; j < n; ++j) buf[j] = b[j];
  int64_t sb = sum_sq_counts(buf, n);
  for (int64_t j = 0; j < n; ++j) buf[j] = pair_key(a[j], b[j]);
  int64_t sab = sum_sq_counts(buf, n);
  return sa + sb - 2 * sab;
}

int mccref_mirkin(const int32_t* a, const int32_t* b, int64_t n, int64_t* result) {
  if (!result || n < 0 || (n > 0 && (!a || !b))) return MCCREF_EINVAL;
  if (!labels_ok(a, n) || !labels_ok(b, n)) return MCCREF_EINVAL;
  if (n == 0) { *result = 0; return 0; }
  int64_t* buf = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!buf) return MCCREF_ENOMEM;
  *result = mirkin_plain(a, b, n, buf);
  free(buf);
  return 0;
}

/* O(C) = sum_i Mirkin(C, P_i)  (Eq. objective1). */
static int64_t objective_plain(const int32_t* c, const int32_t* labels, int32_t k, int64_t n,
                               int64_t* buf) {
  int64_t total = 0;
  for (int32_t i = 0; i < k; ++i) total += mirkin_plain(c, labels + (int64_t)i * n, n, buf);
  return total;
}

int mccref_objective(const int32_t* c, const int32_t* labels, int32_t k, int64_t n,
                     int64_t* result) {
  if (!result || n < 0 || k < 1 || (n > 0 && (!c || !labels))) return MCCREF_EINVAL;
  if (!labels_ok(c, n) || !labels_ok(labels, (int64_t)k * n)) return MCCREF_EINVAL;
  if (n == 0) { *result = 0; return 0; }
  int64_t* buf = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!buf) return MCCREF_ENOMEM;
  *result = objective_plain(c, labels, k, n, buf);
  free(buf);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Counts of the current consensus, rebuilt from scratch                      */
/* ------------------------------------------------------------------------ */
/* For each partition i, the sorted multiset of (C(v), l_i(v)) pairs: the
 * number of copies of (x, l) is N_i(x, l), the number of members of
 * consensus cluster x that P_i puts in cluster l.  size[x] = |x|. */
typedef struct {
  int32_t k;
  int64_t n;
  int64_t* pairs; /* k * n, partition i at pairs + i * n, each sorted */
  int64_t* size;  /* n, indexed by cluster id */
} counts;

static void counts_build(counts* t, const int32_t* c, const int32_t* labels) {
  for (int32_t i = 0; i < t->k; ++i) {
    int64_t* p = t->pairs + (int64_t)i * t->n;
    const int32_t* li = labels + (int64_t)i * t->n;
    for (int64_t v = 0; v < t->n; ++v) p[v] = pair_key(c[v], li[v]);
    qsort(p, (size_t)t->n, sizeof(int64_t), cmp_i64);
  }
  memset(t->size, 0, (size_t)t->n * sizeof(int64_t));
  for (int64_t v = 0; v < t->n; ++v) t->size[c[v]] += 1;
}

/* S_x(v) = sum_i N_i(x, l_i(v)): the (member, partition) pairs of cluster x
 * that agree with v.  Includes v itself when x = C(v). */
static int64_t agree(const counts* t, const int32_t* labels, int64_t v, int32_t x) {
  int64_t s = 0;
  for (int32_t i = 0; i < t->k; ++i)
    s += count_in_sorted(t->pairs + (int64_t)i * t->n, t->n,
                         pair_key(x, labels[(int64_t)i * t->n + v]));
  return s;
}

/* Gain of moving v from c = C(v) to x != c.  Eq. objective3 sums
 * (k - 2 delta_uv) over the members u of c minus the same over the members
 * of x.  With delta_uv = k - (agreements of u and v), summing over the
 * members of a cluster y gives sum_u (k - 2 delta_uv) = 2 S_y(v) - k |y|.
 * The u = v term (k) is removed from the c sum unless `literal` asks for the
 * printed form, which keeps it. */
static int64_t gain(const counts* t, const int32_t* labels, const int32_t* c, int64_t v,
                    int32_t x, int64_t s_own, int literal) {
  int32_t cv = c[v];
  int64_t k = t->k;
  int64_t sum_c = 2 * s_own - k * t->size[cv];   /* over u in c, u = v included */
  int64_t sum_x = 2 * agree(t, labels, v, x) - k * t->size[x];
  int64_t d = sum_c - sum_x;
  if (!literal) d -= k; /* drop the pair (v, v): delta_vv = 0, so its term is k */
  return d;
}

int mccref_delta(const int32_t* c, const int32_t* labels, int32_t k, int64_t n, int64_t v,
                 int32_t target, int64_t* result) {
  if (!c || !labels || !result || k < 1 || n < 1 || v < 0 || v >= n) return MCCREF_EINVAL;
  if (target < 0 || target >= n || target == c[v]) return MCCREF_EINVAL;
  counts t = {k, n, NULL, NULL};
  t.pairs = (int64_t*)malloc((size_t)k * (size_t)n * sizeof(int64_t));
  t.size = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!t.pairs || !t.size) { free(t.pairs); free(t.size); return MCCREF_ENOMEM; }
  counts_build(&t, c, labels);
  *result = gain(&t, labels, c, v, target, agree(&t, labels, v, c[v]), 0);
  free(t.pairs);
  free(t.size);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Best move of one vertex (Eq. objective4)                                  */
/* ------------------------------------------------------------------------ */
/* Candidates are the clusters holding a graph neighbour of v, other than
 * v's own; self-loops are ignored and repeated clusters counted once.  The
 * argmin is over (gain, cluster id), so ties go to the smallest id.
 * dir > 0 keeps only candidates with ids above C(v), dir < 0 only those
 * below (the direction-alternation ablation); dir = 0 keeps all. */
static void score_vertex(const int64_t* row_ptr, const int32_t* col, const int32_t* labels,
                         const int32_t* c, const counts* t, int64_t v, int literal, int dir,
                         int32_t* scratch, int32_t* best, int64_t* dbest, int32_t* ncand) {
  int32_t cv = c[v];
  int64_t m = 0;
  for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
    int32_t u = col[j];
    if (u == v || c[u] == cv) continue;
    if ((dir > 0 && c[u] < cv) || (dir < 0 && c[u] > cv)) continue;
    scratch[m++] = c[u];
  }
  qsort(scratch, (size_t)m, sizeof(int32_t), cmp_i32);
  int64_t distinct = 0;
  for (int64_t j = 0; j < m; ++j)
    if (j == 0 || scratch[j] != scratch[j - 1]) scratch[distinct++] = scratch[j];
  *ncand = (int32_t)distinct;
  *best = -1;
  *dbest = 0;
  if (distinct == 0) return;
  int64_t s_own = agree(t, labels, v, cv);
  for (int64_t j = 0; j < distinct; ++j) {
    int64_t d = gain(t, labels, c, v, scratch[j], s_own, literal);
    if (j == 0 || d < *dbest) { /* ascending ids: strict < keeps the smallest */
      *dbest = d;
      *best = scratch[j];
    }
  }
}

static int64_t max_degree(const int64_t* row_ptr, int64_t n) {
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] - row_ptr[v] > m) m = row_ptr[v + 1] - row_ptr[v];
  return m;
}

static int common_args_ok(const int64_t* row_ptr, const int32_t* col, int64_t n,
                          const int32_t* labels, int32_t k) {
  if (n < 0 || k < 1) return MCCREF_EINVAL;
  if (n == 0) return 0;
  if (!row_ptr || !labels || (row_ptr[n] > 0 && !col)) return MCCREF_EINVAL;
  if ((int64_t)k * n >= ((int64_t)1 << 31)) return MCCREF_EINVAL;
  if (!labels_ok(labels, (int64_t)k * n)) return MCCREF_EINVAL;
  if (!csr_ok(row_ptr, col, n)) return MCCREF_EGRAPH;
  return 0;
}

int mccref_score(const int64_t* row_ptr, const int32_t* col, int64_t n, const int32_t* labels,
                 int32_t k, const int32_t* c, int64_t v_begin, int64_t v_end,
                 int32_t literal_self_term, int32_t* best, int64_t* dbest, int32_t* ncand) {
  int rc = common_args_ok(row_ptr, col, n, labels, k);
  if (rc) return rc;
  if (n == 0 || !c || !best || !dbest || !ncand) return MCCREF_EINVAL;
  if (v_begin < 0 || v_end > n || v_begin > v_end) return MCCREF_EINVAL;
  for (int64_t v = 0; v < n; ++v)
    if (c[v] < 0 || c[v] >= n) return MCCREF_EINVAL;
  counts t = {k, n, NULL, NULL};
  t.pairs = (int64_t*)malloc((size_t)k * (size_t)n * sizeof(int64_t));
  t.size = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* scratch = (int32_t*)malloc((size_t)(max_degree(row_ptr, n) + 1) * sizeof(int32_t));
  if (!t.pairs || !t.size || !scratch) {
    free(t.pairs); free(t.size); free(scratch);
    return MCCREF_ENOMEM;
  }
  counts_build(&t, c, labels);
  for (int64_t v = v_begin; v < v_end; ++v)
    score_vertex(row_ptr, col, labels, c, &t, v, literal_self_term, 0, scratch,
                 best + (v - v_begin), dbest + (v - v_begin), ncand + (v - v_begin));
  free(t.pairs);
  free(t.size);
  free(scratch);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The consensus                                                              */
/* ------------------------------------------------------------------------ */
static int32_t distinct_count(const int32_t* c, int64_t n, int32_t* seen_buf) {
  /* seen_buf: n entries, cluster ids are in [0, n) */
  memset(seen_buf, 0, (size_t)n * sizeof(int32_t));
  int32_t d = 0;
  for (int64_t v = 0; v < n; ++v)
    if (!seen_buf[c[v]]) { seen_buf[c[v]] = 1; ++d; }
  return d;
}

/* (gain, vertex) pairs ordered lexicographically */
static int pair_less(int64_t d1, int64_t w1, int64_t d2, int64_t w2) {
  return d1 < d2 || (d1 == d2 && w1 < w2);
}

int mccref_consensus(const int64_t* row_ptr, const int32_t* col, int64_t n,
                     const int32_t* labels, int32_t k, const int32_t* init, int32_t* out,
                     mccref_stats* stats, int64_t* trace) {
  int rc = common_args_ok(row_ptr, col, n, labels, k);
  if (rc) return rc;
  if (n > 0 && !out) return MCCREF_EINVAL;
  if (init)
    for (int64_t v = 0; v < n; ++v)
      if (init[v] < 0 || init[v] >= n) return MCCREF_EINVAL;
  int32_t max_rounds = (stats && stats->max_rounds > 0) ? stats->max_rounds : 1000;
  int literal = stats ? stats->literal_self_term : 0;
  mccref_stats st;
  memset(&st, 0, sizeof st);
  st.max_rounds = max_rounds;
  st.literal_self_term = literal;
  if (n == 0) {
    st.passes = 1;
    st.converged = 1;
    if (stats) *stats = st;
    return 0;
  }

  counts t = {k, n, NULL, NULL};
  t.pairs = (int64_t*)malloc((size_t)k * (size_t)n * sizeof(int64_t));
  t.size = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* C = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* CA = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* best = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* dbest = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* ncand = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* own_d = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* own_w = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* buf = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* scratch = (int32_t*)malloc((size_t)(max_degree(row_ptr, n) + 1) * sizeof(int32_t));
  if (!t.pairs || !t.size || !C || !CA || !best || !dbest || !ncand || !own_d || !own_w ||
      !buf || !scratch) {
    rc = MCCREF_ENOMEM;
    goto done;
  }

  /* Initialisation: the given partition, or singletons (Methods, "The
   * algorithm"). */
  for (int64_t v = 0; v < n; ++v) C[v] = init ? init[v] : (int32_t)v;
  int64_t O = objective_plain(C, labels, k, n, buf);
  st.objective_init = O;

  for (;;) {
    /* Every vertex finds its best move against the partition as it stands
     * at the start of the pass (Methods, "Parallel algorithm"). */
    counts_build(&t, C, labels);
    for (int64_t v = 0; v < n; ++v)
      score_vertex(row_ptr, col, labels, C, &t, v, literal, 0, scratch, &best[v], &dbest[v],
                   &ncand[v]);
    st.passes += 1;
    int64_t accepted = 0;
    for (int64_t v = 0; v < n; ++v) {
      st.candidate_evals += ncand[v];
      if (ncand[v] > 0 && dbest[v] < 0) ++accepted;
    }
    if (accepted == 0) { /* no vertex can be moved: stop */
      st.converged = 1;
      if (trace) {
        int64_t* r = trace + (int64_t)(st.passes - 1) * 4;
        r[0] = 0; r[1] = 0; r[2] = 0; r[3] = O;
      }
      break;
    }

    /* Validation of the batch: apply every accepted move at once and keep
     * the result only if the objective went down. */
    int64_t committed = 0;
    int fell_back = 0;
    for (int64_t v = 0; v < n; ++v) CA[v] = (ncand[v] > 0 && dbest[v] < 0) ? best[v] : C[v];
    int64_t O_all = objective_plain(CA, labels, k, n, buf);
    if (O_all < O) {
      memcpy(C, CA, (size_t)n * sizeof(int32_t));
      O = O_all;
      committed = accepted;
    } else {
      /* Otherwise each cluster touched by an accepted move (as source or
       * target) is owned by its smallest (gain, vertex) mover, and only the
       * moves owning both of their clusters are applied. */
      fell_back = 1;
      st.fallback_rounds += 1;
      for (int64_t x = 0; x < n; ++x) { own_d[x] = INT64_MAX; own_w[x] = INT64_MAX; }
      for (int64_t w = 0; w < n; ++w) {
        if (!(ncand[w] > 0 && dbest[w] < 0)) continue;
        int32_t xs[2] = {C[w], best[w]};
        for (int e = 0; e < 2; ++e)
          if (pair_less(dbest[w], w, own_d[xs[e]], own_w[xs[e]])) {
            own_d[xs[e]] = dbest[w];
            own_w[xs[e]] = w;
          }
      }
      memcpy(CA, C, (size_t)n * sizeof(int32_t));
      for (int64_t v = 0; v < n; ++v) {
        if (!(ncand[v] > 0 && dbest[v] < 0)) continue;
        if (own_d[C[v]] == dbest[v] && own_w[C[v]] == v && own_d[best[v]] == dbest[v] &&
            own_w[best[v]] == v) {
          CA[v] = best[v];
          ++committed;
        }
      }
      memcpy(C, CA, (size_t)n * sizeof(int32_t));
      O = objective_plain(C, labels, k, n, buf);
    }
    st.moves += committed;
    if (trace) {
      int64_t* r = trace + (int64_t)(st.passes - 1) * 4;
      r[0] = accepted;
      r[1] = committed;
      r[2] = fell_back;
      r[3] = O;
    }
    if (st.passes >= max_rounds) {
      st.converged = 0;
      break;
    }
  }

  memcpy(out, C, (size_t)n * sizeof(int32_t));
  st.objective = O;
  st.clusters = distinct_count(C, n, CA);
  if (stats) *stats = st;
  rc = 0;

done:
  free(t.pairs); free(t.size); free(C); free(CA); free(best); free(dbest); free(ncand);
  free(own_d); free(own_w); free(buf); free(scratch);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Round-rule ablations                                                       */
/* ------------------------------------------------------------------------ */
int mccref_consensus_rule(const int64_t* row_ptr, const int32_t* col, int64_t n,
                          const int32_t* labels, int32_t k, const int32_t* init,
                          int32_t* out, mccref_stats* stats, int64_t* trace, int32_t rule) {
  if (rule == MCCREF_RULE_PINNED)
    return mccref_consensus(row_ptr, col, n, labels, k, init, out, stats, trace);
  if (rule != MCCREF_RULE_ONE_BEST && rule != MCCREF_RULE_ALTERNATE &&
      rule != MCCREF_RULE_UNCHECKED)
    return MCCREF_EINVAL;
  int rc = common_args_ok(row_ptr, col, n, labels, k);
  if (rc) return rc;
  if (n > 0 && !out) return MCCREF_EINVAL;
  if (init)
    for (int64_t v = 0; v < n; ++v)
      if (init[v] < 0 || init[v] >= n) return MCCREF_EINVAL;
  int32_t max_rounds = (stats && stats->max_rounds > 0) ? stats->max_rounds : 1000;
  int literal = stats ? stats->literal_self_term : 0;
  mccref_stats st;
  memset(&st, 0, sizeof st);
  st.max_rounds = max_rounds;
  st.literal_self_term = literal;
  if (n == 0) {
    st.passes = 1;
    st.converged = 1;
    if (stats) *stats = st;
    return 0;
  }

  counts t = {k, n, NULL, NULL};
  t.pairs = (int64_t*)malloc((size_t)k * (size_t)n * sizeof(int64_t));
  t.size = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* C = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* best = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* dbest = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* ncand = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* buf = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* scratch = (int32_t*)malloc((size_t)(max_degree(row_ptr, n) + 1) * sizeof(int32_t));
  if (!t.pairs || !t.size || !C || !best || !dbest || !ncand || !buf || !scratch) {
    rc = MCCREF_ENOMEM;
    goto done;
  }

  for (int64_t v = 0; v < n; ++v) C[v] = init ? init[v] : (int32_t)v;
  int64_t O = objective_plain(C, labels, k, n, buf);
  st.objective_init = O;
  int32_t empty_run = 0; /* consecutive passes without an accepted move */

  for (;;) {
    /* direction of this pass under ALTERNATE: up on even passes */
    int dir = rule == MCCREF_RULE_ALTERNATE ? (st.passes % 2 == 0 ? 1 : -1) : 0;
    counts_build(&t, C, labels);
    for (int64_t v = 0; v < n; ++v)
      score_vertex(row_ptr, col, labels, C, &t, v, literal, dir, scratch, &best[v], &dbest[v],
                   &ncand[v]);
    st.passes += 1;
    int64_t accepted = 0, pick = -1;
    for (int64_t v = 0; v < n; ++v) {
      st.candidate_evals += ncand[v];
      if (!(ncand[v] > 0 && dbest[v] < 0)) continue;
      ++accepted;
      if (pick < 0 || pair_less(dbest[v], v, dbest[pick], pick)) pick = v;
    }
    int64_t committed = 0;
    if (accepted > 0) {
      if (rule == MCCREF_RULE_ONE_BEST) {
        C[pick] = best[pick];
        committed = 1;
      } else {
        /* every accepted move at once, from the frozen state: best[] was
         * computed before any C changes */
        for (int64_t v = 0; v < n; ++v)
          if (ncand[v] > 0 && dbest[v] < 0) C[v] = best[v];
        committed = accepted;
      }
      O = objective_plain(C, labels, k, n, buf);
      empty_run = 0;
    } else {
      empty_run += 1;
    }
    st.moves += committed;
    if (trace) {
      int64_t* r = trace + (int64_t)(st.passes - 1) * 4;
      r[0] = accepted;
      r[1] = committed;
      r[2] = 0;
      r[3] = O;
    }
    /* no improving move left: one empty pass, or under ALTERNATE one empty
     * pass in each direction */
    if (empty_run >= (rule == MCCREF_RULE_ALTERNATE ? 2 : 1)) {
      st.converged = 1;
      break;
    }
    if (st.passes >= max_rounds) {
      st.converged = 0;
      break;
    }
  }

  memcpy(out, C, (size_t)n * sizeof(int32_t));
  st.objective = O;
  st.clusters = distinct_count(C, n, best);
  if (stats) *stats = st;
  rc = 0;

done:
  free(t.pairs); free(t.size); free(C); free(best); free(dbest); free(ncand); free(buf);
  free(scratch);
  return rc;
}

int mccref_canonicalize(const int32_t* in, int32_t* out, int64_t n, int32_t* clusters) {
  if (n < 0 || (n > 0 && (!in || !out))) return MCCREF_EINVAL;
  for (int64_t v = 0; v < n; ++v)
    if (in[v] < 0 || in[v] >= n) return MCCREF_EINVAL;
  int32_t* map = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!map) return MCCREF_ENOMEM;
  for (int64_t x = 0; x < n; ++x) map[x] = -1;
  int32_t next = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (map[in[v]] < 0) map[in[v]] = next++;
    out[v] = map[in[v]];
  }
  if (clusters) *clusters = next;
  free(map);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Partition comparison (Results, "Evaluation metrics")                      */
/* ------------------------------------------------------------------------ */
/* Sum over runs of equal values in the sorted keys of f(run length). */
static double sum_runs_xlogx(const int64_t* keys, int64_t n) {
  double total = 0.0;
  int64_t run = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j > 0 && keys[j] != keys[j - 1]) {
      total += (double)run * log((double)run);
      run = 0;
    }
    ++run;
  }
  if (n > 0) total += (double)run * log((double)run);
  return total;
}

static int32_t count_runs(const int64_t* keys, int64_t n) {
  int32_t runs = 0;
  for (int64_t j = 0; j < n; ++j)
    if (j == 0 || keys[j] != keys[j - 1]) ++runs;
  return runs;
}

/* Keys (x, y) sorted: sum over x of the largest count of one (x, y) pair. */
static int64_t sum_of_row_maxima(const int64_t* keys, int64_t n) {
  int64_t total = 0, best = 0, run = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j > 0 && keys[j] != keys[j - 1]) {
      if (run > best) best = run;
      run = 0;
      if ((keys[j] >> 32) != (keys[j - 1] >> 32)) { /* next row */
        total += best;
        best = 0;
      }
    }
    ++run;
  }
  if (n > 0) {
    if (run > best) best = run;
    total += best;
  }
  return total;
}

static void compare_plain(const int32_t* a, const int32_t* b, int64_t n, int64_t* buf,
                          mccref_comparison* r) {
  memset(r, 0, sizeof *r);
  if (n == 0) return;
  r->mirkin = mirkin_plain(a, b, n, buf);
  /* cluster sizes and sum |A| ln |A|, sum |B| ln |B| */
  for (int64_t j = 0; j < n; ++j) buf[j] = a[j];
  qsort(buf, (size_t)n, sizeof(int64_t), cmp_i64);
  const double ha = sum_runs_xlogx(buf, n);
  r->clusters_a = count_runs(buf, n);
  for (int64_t j = 0; j < n; ++j) buf[j] = b[j];
  qsort(buf, (size_t)n, sizeof(int64_t), cmp_i64);
  const double hb = sum_runs_xlogx(buf, n);
  r->clusters_b = count_runs(buf, n);
  /* intersections, grouped by the cluster of a, then by the cluster of b */
  for (int64_t j = 0; j < n; ++j) buf[j] = pair_key(a[j], b[j]);
  qsort(buf, (size_t)n, sizeof(int64_t), cmp_i64);
  const double hab = sum_runs_xlogx(buf, n);
  r->split_join_ab = n - sum_of_row_maxima(buf, n);
  for (int64_t j = 0; j < n; ++j) buf[j] = pair_key(b[j], a[j]);
  qsort(buf, (size_t)n, sizeof(int64_t), cmp_i64);
  r->split_join_ba = n - sum_of_row_maxima(buf, n);
  r->split_join = r->split_join_ab + r->split_join_ba;
  /* VI = H(A) + H(B) - 2 I(A; B) = (sum |A| ln|A| + sum |B| ln|B|
   *      - 2 sum |A n B| ln|A n B|) / n */
  r->vi = (ha + hb - 2.0 * hab) / (double)n;
  r->rand = n > 1 ? (double)r->mirkin / ((double)n * (double)(n - 1)) : 0.0;
}

int mccref_compare(const int32_t* a, const int32_t* b, int64_t n, mccref_comparison* r) {
  if (!r || n < 0 || (n > 0 && (!a || !b))) return MCCREF_EINVAL;
  if (!labels_ok(a, n) || !labels_ok(b, n)) return MCCREF_EINVAL;
  int64_t* buf = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!buf) return MCCREF_ENOMEM;
  compare_plain(a, b, n, buf, r);
  free(buf);
  return 0;
}

int mccref_split_join_matrix(const int32_t* labels, int32_t k, int64_t n, int64_t* dist) {
  if (!dist || k < 1 || n < 0 || (n > 0 && !labels)) return MCCREF_EINVAL;
  if (!labels_ok(labels, (int64_t)k * n)) return MCCREF_EINVAL;
  int64_t* buf = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!buf) return MCCREF_ENOMEM;
  for (int32_t i = 0; i < k; ++i) {
    dist[(int64_t)i * k + i] = 0;
    for (int32_t j = i + 1; j < k; ++j) {
      mccref_comparison r;
      compare_plain(labels + (int64_t)i * n, labels + (int64_t)j * n, n, buf, &r);
      dist[(int64_t)i * k + j] = r.split_join;
      dist[(int64_t)j * k + i] = r.split_join;
    }
  }
  free(buf);
  return 0;
}

/* Components of the graph on k partitions with an edge where the distance
 * is at most lambda: a plain depth-first search from each unvisited
 * partition in increasing order. */
static int32_t components(const int64_t* dist, int32_t k, int64_t lambda, int32_t* group,
                          int32_t* stack) {
  int32_t ng = 0;
  for (int32_t i = 0; i < k; ++i) group[i] = -1;
  for (int32_t s = 0; s < k; ++s) {
    if (group[s] >= 0) continue;
    int32_t top = 0;
    stack[top++] = s;
    group[s] = ng;
    while (top > 0) {
      const int32_t u = stack[--top];
      for (int32_t w = 0; w < k; ++w)
        if (group[w] < 0 && dist[(int64_t)u * k + w] <= lambda) {
          group[w] = ng;
          stack[top++] = w;
        }
    }
    ++ng;
  }
  return ng;
}

int mccref_group(const int64_t* dist, int32_t k, int64_t lambda, int32_t* group,
                 int32_t* ngroups) {
  if (!dist || !group || !ngroups || k < 1) return MCCREF_EINVAL;
  int32_t* stack = (int32_t*)malloc((size_t)k * sizeof(int32_t));
  if (!stack) return MCCREF_ENOMEM;
  *ngroups = components(dist, k, lambda, group, stack);
  free(stack);
  return 0;
}

int mccref_elbow_lambda(const int64_t* dist, int32_t k, int64_t* lambda) {
  if (!dist || !lambda || k < 1) return MCCREF_EINVAL;
  *lambda = 0;
  if (k < 2) return 0;
  const int64_t m_all = (int64_t)k * (k - 1) / 2;
  int64_t* t = (int64_t*)malloc((size_t)m_all * sizeof(int64_t));
  int32_t* group = (int32_t*)malloc((size_t)k * sizeof(int32_t));
  int32_t* stack = (int32_t*)malloc((size_t)k * sizeof(int32_t));
  if (!t || !group || !stack) {
    free(t); free(group); free(stack);
    return MCCREF_ENOMEM;
  }
  int64_t m = 0;
  for (int32_t i = 0; i < k; ++i)
    for (int32_t j = i + 1; j < k; ++j) t[m++] = dist[(int64_t)i * k + j];
  qsort(t, (size_t)m, sizeof(int64_t), cmp_i64);
  int64_t d = 0; /* distinct values */
  for (int64_t j = 0; j < m; ++j)
    if (j == 0 || t[j] != t[d - 1]) t[d++] = t[j];
  *lambda = t[0];
  if (d >= 3) {
    const double g0 = components(dist, k, t[0], group, stack);
    const double g1 = components(dist, k, t[d - 1], group, stack);
    if (g0 != g1) {
      double best = 0.0;
      for (int64_t j = 0; j < d; ++j) {
        const double x = (double)(t[j] - t[0]) / (double)(t[d - 1] - t[0]);
        const double y = (components(dist, k, t[j], group, stack) - g1) / (g0 - g1);
        const double below = 1.0 - x - y; /* distance below the chord, up to a factor */
        if (below > best) {
          best = below;
          *lambda = t[j];
        }
      }
    }
  }
  free(t); free(group); free(stack);
  return 0;
}
