/*
 * mccref: plain sequential CPU oracle for median consensus clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  This code defines the expected result of the
 * GPU library; it is called by the tests, by the package's smoke check and
 * by the benchmark's CPU-baseline leg, never by the product path.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Paper: "Parallel Algorithms for Median Consensus Clustering in Complex
 * Networks" (Hussain, Halappanavar, Chatterjee, Radicchi, Fortunato, Azad).
 *
 * All pointers are HOST pointers.  Labels are one contiguous partition-major
 * array: labels[i * n + v] is the cluster of vertex v in input partition i.
 * Any label value >= 0 is allowed.  Graphs are CSR: row_ptr[n + 1] (int64),
 * col[nnz] (int32); arcs are read as given (self-loops ignored, duplicate
 * arcs harmless).
 *
 * Return codes: 0 success, MCCREF_EINVAL bad argument, MCCREF_EGRAPH bad
 * CSR, MCCREF_ENOMEM allocation failure.
 */
#ifndef MCCREF_H
#define MCCREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCCREF_EINVAL (-1)
#define MCCREF_EGRAPH (-2)
#define MCCREF_ENOMEM (-3)

typedef struct {
  /* in */
  int32_t max_rounds;        /* cap on scoring passes; 0 means 1000 */
  int32_t literal_self_term; /* 1: score with the paper's printed sum over all
                                u including u = v (adds k to every gain);
                                0: exact gain (default) */
  /* out */
  int32_t passes;            /* scoring passes run, including the last one
                                that finds no improving move */
  int32_t converged;         /* 1 if stopped because no vertex can move */
  int32_t fallback_rounds;   /* passes whose full batch did not lower O */
  int32_t clusters;          /* distinct clusters in the output */
  int64_t moves;             /* committed vertex moves, all passes */
  int64_t candidate_evals;   /* sum over passes and vertices of |cand(v)| */
  int64_t objective_init;    /* O(init) = sum_i Mirkin(init, P_i) */
  int64_t objective;         /* O(out) */
} mccref_stats;

/* Mirkin distance between partitions a and b of n items: the number of
 * ordered pairs (u, v), u != v, co-clustered in exactly one of them
 * (Methods, "The consensus clustering problem"; Appendix, Eq. distance,
 * counted over ordered pairs). */
int mccref_mirkin(const int32_t* a, const int32_t* b, int64_t n, int64_t* result);

/* O(C) = sum_i Mirkin(C, P_i)  (Eq. objective1 with the Mirkin distance). */
int mccref_objective(const int32_t* c, const int32_t* labels, int32_t k, int64_t n,
                     int64_t* result);

/* Exact gain of moving v from C(v) to cluster `target` (Eq. objective3 with
 * the u = v term left out), in unordered-pair units:
 * O(after) - O(before) = 2 * result. */
int mccref_delta(const int32_t* c, const int32_t* labels, int32_t k, int64_t n,
                 int64_t v, int32_t target, int64_t* result);

/* Best move of each vertex in [v_begin, v_end) against the frozen state c
 * (Eq. objective4): best[j] = argmin over neighbour clusters of (gain, id),
 * or -1 when v has no candidate; dbest[j] its gain (0 if none); ncand[j] the
 * number of candidate clusters.  Arrays are indexed j = v - v_begin. */
int mccref_score(const int64_t* row_ptr, const int32_t* col, int64_t n,
                 const int32_t* labels, int32_t k, const int32_t* c,
                 int64_t v_begin, int64_t v_end, int32_t literal_self_term,
                 int32_t* best, int64_t* dbest, int32_t* ncand);

/* The whole greedy consensus with synchronous rounds (Methods, "The
 * algorithm" and "Parallel algorithm").  init: int32[n] in [0, n), used
 * verbatim as cluster IDs, or NULL for singletons.  out: int32[n], may alias
 * init.  trace: NULL or int64[max_rounds * 4] receiving per pass
 * (accepted, committed, fallback, objective after the pass); the final
 * pass that finds no move records (0, 0, 0, O). */
int mccref_consensus(const int64_t* row_ptr, const int32_t* col, int64_t n,
                     const int32_t* labels, int32_t k, const int32_t* init,
                     int32_t* out, mccref_stats* stats, int64_t* trace);

/* ---- round-rule ablations (Methods, "Parallel algorithm") -------------- */
/* The paper applies every vertex's best move together and notes that the
 * sequential alternative, one best move per iteration, converges to the same
 * quality in fewer moves per iteration; it leaves its validation checks
 * unspecified.  These rules run on the same scoring as mccref_consensus:
 *
 *   MCCREF_RULE_PINNED     the rule of mccref_consensus (batch, validated,
 *                          conflict-free fallback).
 *   MCCREF_RULE_ONE_BEST   every pass scores all vertices, then applies only
 *                          the smallest (gain, vertex) accepted move.
 *   MCCREF_RULE_ALTERNATE  even passes allow moves only to larger cluster ids,
 *                          odd passes only to smaller ones; the batch is
 *                          applied unchecked; the solve stops after two
 *                          consecutive passes without a move (one in each
 *                          direction), i.e. when no improving move is left.
 *   MCCREF_RULE_UNCHECKED  the batch is applied unchecked (may oscillate;
 *                          converged = 0 at the pass cap).
 *
 * Arguments, stats and trace as for mccref_consensus; the trace's third
 * column is the fallback flag under the pinned rule, 0 otherwise.
 * candidate_evals counts the candidates scored (under ALTERNATE, those in
 * the pass's direction). */
#define MCCREF_RULE_PINNED 0
#define MCCREF_RULE_ONE_BEST 1
#define MCCREF_RULE_ALTERNATE 2
#define MCCREF_RULE_UNCHECKED 3
int mccref_consensus_rule(const int64_t* row_ptr, const int32_t* col, int64_t n,
                          const int32_t* labels, int32_t k, const int32_t* init,
                          int32_t* out, mccref_stats* stats, int64_t* trace, int32_t rule);

/* Relabel cluster ids in [0, n) to [0, clusters) in order of first occurrence. */
int mccref_canonicalize(const int32_t* in, int32_t* out, int64_t n, int32_t* clusters);

/* ---- partition comparison (Results, "Evaluation metrics") ------------- */
typedef struct {
  int64_t mirkin;        /* ordered pairs co-clustered in exactly one of a, b */
  int64_t split_join_ab; /* n - sum over clusters A of max_B |A n B| */
  int64_t split_join_ba; /* n - sum over clusters B of max_A |A n B| */
  int64_t split_join;    /* their sum: the split-join (projection) distance */
  double rand;           /* Rand distance: mirkin / (n (n - 1)); 0 if n < 2 */
  double vi;             /* variation of information, natural logarithm */
  int32_t clusters_a, clusters_b;
} mccref_comparison;

int mccref_compare(const int32_t* a, const int32_t* b, int64_t n, mccref_comparison* r);

/* dist[i * k + j] = split-join distance between partitions i and j (the
 * edge weights of the grouping step, Methods, "Grouping homogeneous
 * partitions").  labels as for mccref_consensus. */
int mccref_split_join_matrix(const int32_t* labels, int32_t k, int64_t n, int64_t* dist);

/* Groups of homogeneous partitions: i and j are linked when
 * dist[i * k + j] <= lambda; the groups are the connected components,
 * numbered 0, 1, ... in order of their smallest member. */
int mccref_group(const int64_t* dist, int32_t k, int64_t lambda, int32_t* group,
                 int32_t* ngroups);

/* The threshold by the elbow rule: over the distinct pairwise distances t
 * in increasing order, the number of groups g(t) falls; with both axes
 * scaled to [0, 1] between the first and last point, the elbow is the t
 * farthest below the straight line joining them (first such t on ties).
 * Fewer than three distinct distances, or a flat curve: the smallest
 * distance (0 when k < 2). */
int mccref_elbow_lambda(const int64_t* dist, int32_t k, int64_t* lambda);

#ifdef __cplusplus
}
#endif
#endif
