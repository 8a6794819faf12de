/*
 * libmcc: median consensus clustering on AMD Instinct MI355X (gfx950).
 *
 * Method: "Parallel Algorithms for Median Consensus Clustering in Complex
 * Networks" (Hussain, Halappanavar, Chatterjee, Radicchi, Fortunato, Azad).
 * Given a graph and k partitions P_1..P_k of its vertices, find a consensus
 * partition C minimising sum_i Mirkin(C, P_i) (Eq. objective1) by greedy
 * local moves: each vertex may move into a cluster that holds one of its
 * graph neighbours (Eq. objective4), scored by the exact change of the
 * objective (Eq. objective3 without the vertex's pair with itself), all
 * vertices scored against the partition as it stands at the start of a pass
 * and the accepted moves applied together (Methods, "Parallel algorithm").
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (memory on the current HIP device,
 *    e.g. a torch tensor's data_ptr), unless a comment says "host".  The
 *    caller owns every buffer; the library keeps no pointer to them after a
 *    call returns.  Its own workspace is kept between calls, per device and
 *    shared by the calls of every stream (at most 64 GiB in total;
 *    mcc_release_workspace frees it), so that repeated calls allocate
 *    nothing.  When an allocation fails, the
 *    idle workspace the library keeps on that device (any stream) is freed
 *    and the allocation tried once more before MCC_ENOMEM is returned.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Each call is stream-ordered and returns only once its results
 *    are complete (it synchronises with the stream).
 *  - Return value: 0 on success or a negative MCC_E* code.  No C++
 *    exception crosses this interface.  On error, outputs are unspecified.
 *  - Calls on different streams are independent; calls that share a stream
 *    are serialised by it.
 */
#ifndef MCC_H
#define MCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define MCC_OK 0
#define MCC_EINVAL (-1)   /* NULL pointer, k < 1, n < 0, n*k >= 2^31, a label < 0,
                             an init id outside [0, n), bad sizes */
#define MCC_EGRAPH (-2)   /* invalid CSR (only checked with MCC_F_VALIDATE) */
#define MCC_ENOMEM (-3)   /* device allocation failed */
#define MCC_EDEVICE (-4)  /* a HIP runtime call failed; see mcc_strerror */
#define MCC_ENOTSUP (-5)  /* the instance needs a table larger than the library
                             supports (see mcc_consensus) */
#define MCC_ESCRATCH (-6) /* mcc_consensus_noalloc: the instance needs more
                             workspace than the scratch array holds */

/* Size of the per-device scratch array of mcc_consensus_noalloc, MiB. */
#define MCC_NOALLOC_SCRATCH_MIB 256

/* ---- flags --------------------------------------------------------------- */
#define MCC_F_VALIDATE 0x1u /* check the CSR on the device before solving */
#define MCC_F_TRACE 0x2u    /* fill stats->trace (host array) per pass */
#define MCC_F_LITERAL 0x4u  /* score with the paper's printed Eq. objective3,
                               whose sum over u includes u = v and so adds k to
                               every gain (an ablation; default is the exact
                               gain) */
#define MCC_F_PROFILE 0x8u  /* time every scoring kernel with HIP events on the
                               call's stream (stats->ms_score) */
#define MCC_F_ARC_CACHE 0x10u /* keep a per-arc copy of the neighbour's cluster,
                                 updated through in-arc lists when vertices
                                 move, instead of gathering clusters every
                                 pass (costs nnz * 8 bytes and a list build;
                                 pays off with many passes; a tuning knob,
                                 results do not depend on it) */
#define MCC_F_SYMMETRIC 0x40u /* the caller states that the graph is symmetric
                                 (every arc (v, u) has a reverse arc (u, v)):
                                 candidate sets are then carried over between
                                 passes for vertices with no moved neighbour.
                                 Results do not change; on a graph that is not
                                 symmetric they may differ from the exact
                                 method, so with MCC_F_VALIDATE the library
                                 checks the property (MCC_EGRAPH if it fails) */
#define MCC_F_HASH_TABLES 0x20u /* keep the contingency counts in one
                                   open-addressing hash table even where dense
                                   tables fit (they are chosen automatically
                                   when dense tables would not fit or would be
                                   far larger; results do not depend on it) */
#define MCC_F_HASH_ROWS 0x80u /* hashed tables: use the row layout (keys
                                 (cluster, label id) with the label ids of
                                 every partition aligned to partition 0's,
                                 each key owning a row of k counts) whenever
                                 its indices fit, not only where it is no
                                 larger than the key layout; results do not
                                 depend on it */
#define MCC_F_HASH_KEYS 0x100u /* hashed tables: always use the key layout
                                  (one slot per (cluster, partition, label));
                                  results do not depend on it */

/* CSR graph: row_ptr[n + 1] (int64, row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz) and col[nnz] (int32 vertex ids in [0, n)).  Arcs are
 * read as out-neighbours; self-loops are ignored and repeated arcs are
 * harmless.  Undirected graphs store both directions. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col;
} mcc_csr;

typedef struct {
  /* in */
  int32_t max_rounds; /* cap on scoring passes; 0 means 1000 */
  uint32_t flags;     /* MCC_F_* */
  void* stream;       /* hipStream_t or NULL */
  int64_t* trace;     /* host int64[max_rounds * 4] when MCC_F_TRACE: per pass
                         (accepted moves, committed moves, 1 if the pass fell
                         back to the conflict-free subset, objective after
                         the pass); the final pass that finds no move records
                         (0, 0, 0, objective) */
  int32_t lanes;      /* scoring kernel: 0 = tiled scorer (default), else one
                         of 4, 8, 16, 32, 64 lanes per vertex for the group
                         scorer (a tuning knob; results do not depend on it) */
  int32_t reserved;
  /* out */
  int32_t passes;          /* scoring passes, including the final one that
                              finds no improving move */
  int32_t converged;       /* 1 if stopped because no vertex can move */
  int32_t fallback_rounds; /* passes whose full batch did not lower the
                              objective */
  int32_t clusters;        /* distinct clusters in the output */
  int64_t moves;           /* committed vertex moves over all passes */
  int64_t candidate_evals; /* sum over passes and vertices of the number of
                              candidate clusters scored */
  int64_t objective_init;  /* sum_i Mirkin(init, P_i) */
  int64_t objective;       /* sum_i Mirkin(out, P_i) */
  float ms_total;          /* wall time of the call on the stream */
  float ms_passes;         /* time spent in the pass loop */
  int64_t boundary;        /* sum over passes of the vertices that had at
                              least one candidate (their label rows are read) */
  float ms_score;          /* with MCC_F_PROFILE: summed duration of the
                              scoring kernels of the executed passes */
  int32_t lanes_used;      /* the `lanes` the scoring ran with (0 = tiled) */
  int32_t tables;          /* contingency table layout used: 0 dense blocked,
                              1 dense interleaved, 2 hashed keys, 3 hashed
                              rows */
  int64_t skipped_evals;   /* of candidate_evals, those not recomputed because
                              an exact bound showed the vertex could not
                              propose (with MCC_F_SYMMETRIC; they count in
                              candidate_evals as the method scores them) */
  int64_t workspace_bytes; /* device workspace the call held (kept by the
                              library for later calls on the stream) */
} mcc_stats;

/*
 * Greedy median consensus (Methods, "The algorithm" and "Parallel
 * algorithm").
 *
 *  g       CSR graph (host struct holding device pointers).
 *  labels  HOST array of k device pointers; labels[i] is int32[n] holding
 *          partition P_i (any label values >= 0).
 *  k       number of input partitions, >= 1.
 *  init    int32[n] initial consensus, ids in [0, n) used verbatim as cluster
 *          ids (they are the tie-break keys), or NULL for singletons
 *          (C(v) = v, the paper's initialisation).
 *  out     int32[n] final consensus as cluster ids (a subset of the initial
 *          ids, so passing it back as `init` resumes exactly).  May alias
 *          init.
 *  stats   host struct, may be NULL (then max_rounds = 1000, no flags, the
 *          default stream).
 *
 * Per pass, with the partition frozen: every vertex v scores each cluster c'
 * holding a neighbour (other than its own cluster c) by
 *   gain = 2 (S_c(v) - S_c'(v)) + k (|c'| - |c| - 1),
 *   S_x(v) = sum_i |{u in x : P_i(u) = P_i(v)}|,
 * keeps the smallest (gain, cluster id) and proposes it if gain < 0.  If
 * applying all proposals together lowers the objective they are committed;
 * otherwise each cluster touched by a proposal is owned by its smallest
 * (gain, vertex id) proposer and only proposals owning both of their clusters
 * are committed.  The loop stops when no vertex proposes (converged = 1) or
 * after max_rounds passes (converged = 0, not an error).
 *
 * The result (out and every stats field except the timings) is a
 * deterministic function of the inputs and equals the plain sequential
 * definition bit for bit.  Limits: n * k < 2^31; nnz < 2^31 - 1 (else
 * MCC_ENOTSUP); the contingency tables
 * (consensus cluster x label, per partition) must fit the library's table
 * budget, else MCC_ENOTSUP.
 */
int mcc_consensus(const mcc_csr* g, const int32_t* const* labels, int32_t k,
                  const int32_t* init, int32_t* out, mcc_stats* stats);

/*
 * mcc_consensus for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, hosts that forbid
 * hipMalloc): the same arguments, the same results bit for bit, but the
 * workspace is a static device array of MCC_NOALLOC_SCRATCH_MIB MiB inside
 * the library (each device the library runs on holds its own copy from the
 * library's first use there until the process ends) and the call makes no
 * hipMalloc or hipFree.  Instances whose workspace exceeds the array
 * (roughly 4 n k + 48 n bytes plus the contingency tables) fail with
 * MCC_ESCRATCH before anything is computed, or during set-up when the
 * tables turn out too large; the outputs are then unspecified.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (on different streams
 * or host threads) race and give wrong results; serialise them.
 */
int mcc_consensus_noalloc(const mcc_csr* g, const int32_t* const* labels, int32_t k,
                          const int32_t* init, int32_t* out, mcc_stats* stats);

/*
 * Objective of a given partition: *result (host) = sum_i Mirkin(c, P_i)
 * (Eq. objective1), Mirkin counted over ordered pairs.  c: int32[n] ids in
 * [0, n); labels as for mcc_consensus.
 */
int mcc_objective(const int32_t* c, const int32_t* const* labels, int32_t k, int64_t n,
                  int64_t* result, void* stream);

/*
 * Mirkin distance (Methods, "The consensus clustering problem"; Appendix,
 * Eq. distance): *result (host) = the number of ordered pairs (u, v), u != v,
 * co-clustered in exactly one of a and b = sum |A|^2 + sum |B|^2
 * - 2 sum |A n B|^2.  a, b: int32[n], any label values >= 0.
 */
int mcc_mirkin(const int32_t* a, const int32_t* b, int64_t n, int64_t* result, void* stream);

/*
 * Relabel cluster ids in [0, n) to [0, *clusters) in order of first
 * occurrence (presentation labels for a consensus).  in, out: int32[n], may
 * alias.  clusters: host, may be NULL.
 */
int mcc_canonicalize(const int32_t* in, int32_t* out, int64_t n, int32_t* clusters,
                     void* stream);

/* One instance of a batch: the arguments of mcc_consensus.  `labels` is a
 * HOST array of k device pointers. */
typedef struct {
  mcc_csr g;
  const int32_t* const* labels;
  int32_t k;
  const int32_t* init;
  int32_t* out;
} mcc_problem;

/*
 * Launch shape of the batched solver, chosen per size bucket by
 * mcc_batch_tune.  A bucket holds the instances with
 * floor(log2(max(n, 1))) == n_log2 and k in the class k_class
 * (0: k <= 8, 1: k <= 16, 2: k <= 32, 3: k <= 64, 4: k <= 256).
 */
#define MCC_TUNE_LANES 5      /* candidate lanes per vertex: 4, 8, 16, 32, 64 */
#define MCC_TUNE_MAX_BUCKETS 160
typedef struct {
  int32_t n_log2;
  int32_t k_class;
  int32_t lanes;      /* lanes per vertex chosen for the bucket */
  int32_t instances;  /* instances of the bucket the choice was measured on */
  int64_t cells;      /* largest contingency table (int32 cells) seen in it */
  float ms[MCC_TUNE_LANES]; /* summed per-instance device time for each
                               candidate lanes value, in the order above
                               (negative: not measured) */
  int32_t pad;
} mcc_tune_entry;

typedef struct {
  int32_t count;      /* valid entries */
  int32_t wg_per_cu;  /* resident workgroups per compute unit (1..8) */
  mcc_tune_entry entry[MCC_TUNE_MAX_BUCKETS];
} mcc_tune_table;

typedef struct {
  void* stream;       /* hipStream_t or NULL */
  int32_t max_rounds; /* per instance; 0 means 1000 */
  uint32_t flags;     /* MCC_F_LITERAL honoured; others ignored */
  int32_t lanes;      /* lanes per vertex for every instance: 4, 8, 16, 32 or 64;
                         0: per instance from the tune table (`tune`, else
                         the file `tune_cache_path`, else a built-in rule) */
  int32_t wg_per_cu;  /* resident workgroups per compute unit: 0 (= the
                         tune table's, else 2) .. 8 */
  int32_t* status;    /* optional host int32[count]: per-instance return code */
  const mcc_tune_table* tune;  /* optional host pointer, read only */
  const char* tune_cache_path; /* optional text file written by mcc_tune_save */
  int32_t solved_in_batch; /* out: instances the persistent kernel finished
                              (the rest went through mcc_consensus) */
  float ms_total;     /* out: wall time of the call on the stream */
  int64_t workspace_bytes; /* out: device workspace the call held at most
                              (kept by the library for later calls on the
                              stream) */
} mcc_batch_opts;

/*
 * Many independent consensus problems in one persistent launch (the groups
 * of homogeneous partitions the paper solves independently, Methods, "The
 * algorithm").  Each workgroup of the kernel takes one instance at a time
 * from a queue ordered by estimated work (largest first) and runs the whole
 * method of mcc_consensus on it; the launch is captured in a HIP graph.
 * Instances beyond a workgroup's capacities (more than 256 partitions,
 * label values far above n, large contingency tables) are solved by
 * mcc_consensus on the same stream.  Every out[] and every stats field
 * except the timings equals what mcc_consensus returns for the instance.
 *
 *  probs  host array of `count` problems.
 *  stats  host array of `count` stats (outputs only) or NULL.
 *  opts   may be NULL (defaults).
 * Returns 0, or the first nonzero code of an instance (all instances are
 * attempted; per-instance codes go to opts->status when given).
 */
int mcc_consensus_batch(const mcc_problem* probs, int32_t count, mcc_stats* stats,
                        mcc_batch_opts* opts);

/*
 * Autotuner of the batched solver (the many-instance launch above).
 * Solves every problem once per candidate lanes value (4, 8, 16, 32, 64),
 * each time in one persistent launch whose workgroups time their own
 * instances, and keeps for each size bucket the lanes value with the
 * smallest summed time; records per bucket the largest contingency table
 * seen (the workspace table size of later launches); then times whole
 * launches at 1, 2, 4 and 8 resident workgroups per compute unit with the
 * chosen lanes and keeps the fastest, among the values that give every
 * workgroup two or more problems on average (if fewer than two qualify,
 * the table keeps 2).  The problems stand for the workload the table is
 * meant for, at its batch size; their out[] buffers are not written
 * (results go to scratch).  The choice never changes a result: every lanes
 * value computes the same output.
 *
 *  probs, count  as for mcc_consensus_batch (out may be NULL: it is not
 *                used); instances with k > 256 are ignored.
 *  opts          stream, max_rounds and flags are used (may be NULL); if
 *                tune_cache_path is set the table is also written there.
 *  table         host output.
 * Returns 0, MCC_EINVAL (a problem fails the argument checks, table NULL)
 * or the first error of a launch.
 */
int mcc_batch_tune(const mcc_problem* probs, int32_t count, const mcc_batch_opts* opts,
                   mcc_tune_table* table);

/*
 * Device memory budgeting (for callers that admit work by memory, such as
 * a server).  Host only; nothing is launched or allocated.
 *
 * mcc_workspace_bound: an upper bound of the workspace mcc_consensus takes
 * for an instance of n vertices, nnz arcs and k partitions whose label
 * values all lie in [0, max_label], started from an init with `clusters`
 * distinct ids (0: unknown, or singletons), with these flags: every array
 * it sizes from those figures (the contingency tables at the largest size
 * the layouts that can be chosen may take: a hashed row table counts as the
 * key table it may not exceed unless MCC_F_HASH_ROWS is set, plus the
 * alignment to partition 0's labels), arrays below the 16 MiB chunk
 * size counted twice for the chunk ends they may leave unused, plus one
 * chunk.  The exact figure of a finished call is stats->workspace_bytes.
 *
 * mcc_batch_workspace_bytes: the workspace of one mcc_consensus_batch call
 * over these problems and options: the persistent launch's slots as the
 * call would size them (twice over for chunking, plus one chunk), or the
 * bound of the largest instance the call hands to mcc_consensus if that is
 * larger (instances with k > 256; instances that turn out to exceed a
 * slot's table are not foreseen).  The exact figure of a finished call is
 * opts->workspace_bytes.
 *
 * mcc_workspace_held: the workspace the library keeps, between calls, on
 * the current device (0 if none), shared by the calls of every stream: what
 * the library holds there when no call is running.
 *
 * All three return 0 or MCC_EINVAL (NULL bytes, sizes out of range);
 * mcc_workspace_held may return MCC_EDEVICE.
 */
int mcc_workspace_bound(int64_t n, int64_t nnz, int32_t k, int64_t max_label, int64_t clusters,
                        uint32_t flags, int64_t* bytes);
int mcc_batch_workspace_bytes(const mcc_problem* probs, int32_t count,
                              const mcc_batch_opts* opts, int64_t* bytes);
int mcc_workspace_held(int64_t* bytes);

/* Write a tune table as text to `path` / read it back.  Host only.
 * Returns 0, MCC_EINVAL (NULL argument, unreadable or malformed file,
 * values out of range) or MCC_EDEVICE (the file cannot be written). */
int mcc_tune_save(const mcc_tune_table* table, const char* path);
int mcc_tune_load(mcc_tune_table* table, const char* path);

/*
 * Comparison of two partitions of the same n elements (Results, "Evaluation
 * metrics": the paper reports the variation of information, split-join and
 * Rand distances; the first two follow their cited definitions, the last is
 * the Mirkin distance normalised by the n (n - 1) ordered pairs).  With
 * n_ab = |A_a n B_b|, n_a = |A_a|, n_b = |B_b|:
 *   split_join_ab = n - sum_a max_b n_ab,  split_join_ba = n - sum_b max_a n_ab,
 *   split_join    = split_join_ab + split_join_ba (van Dongen's distance),
 *   vi   = (sum_a n_a ln n_a + sum_b n_b ln n_b - 2 sum_ab n_ab ln n_ab) / n,
 *   rand = mirkin / (n (n - 1))  (0 when n < 2).
 * Integers are exact; vi is summed in double precision in a fixed order (the
 * same bits on every call).
 */
typedef struct {
  int64_t mirkin;
  int64_t split_join_ab, split_join_ba, split_join;
  double rand;
  double vi;
  int32_t clusters_a, clusters_b;
} mcc_comparison;

/*  a, b    device int32[n], any values >= 0.
 *  result  host output.
 * Returns 0, MCC_EINVAL (NULL result, n outside [0, 2^31), a negative label,
 * a pointer not visible to the device), MCC_ENOMEM, MCC_EDEVICE. */
int mcc_compare(const int32_t* a, const int32_t* b, int64_t n, mcc_comparison* result,
                void* stream);

/*
 * Split-join distance of every pair of the k partitions (the edge weights
 * of the grouping step, Methods, "Grouping homogeneous partitions"), all
 * pairs counted in one launch.
 *  labels  host array of k device pointers, each int32[n], values >= 0.
 *  dist    host int64[k * k] output, symmetric, zero diagonal.
 * Returns 0, MCC_EINVAL (NULL argument, k < 1, k n >= 2^31, a negative
 * label), MCC_ENOMEM, MCC_EDEVICE.
 */
int mcc_split_join_matrix(const int32_t* const* labels, int32_t k, int64_t n, int64_t* dist,
                          void* stream);

/*
 * Groups of homogeneous partitions (Methods, "Grouping homogeneous
 * partitions"): partitions i and j are linked when dist[i k + j] <= lambda,
 * and the groups are the connected components, numbered 0, 1, ... in order
 * of their smallest member.  lambda < 0 picks it by the elbow rule: over the
 * distinct pairwise distances t in increasing order, with the number of
 * groups g(t) and both axes scaled to [0, 1] between the first and the last
 * distance, the t farthest below the straight line joining those two points
 * (the first on ties); the smallest distance when there are fewer than
 * three distinct distances or g does not change.  Host only.
 *  dist         host int64[k * k], symmetric, >= 0.
 *  group        host int32[k] output; ngroups host output.
 *  lambda_used  host output or NULL: the threshold applied.
 * Returns 0 or MCC_EINVAL (NULL argument, k < 1, dist not symmetric or
 * negative).
 */
int mcc_group_from_distances(const int64_t* dist, int32_t k, int64_t lambda, int32_t* group,
                             int32_t* ngroups, int64_t* lambda_used);

/* The split-join matrix of the partitions (mcc_split_join_matrix) and the
 * groups it gives (mcc_group_from_distances).  dist: host int64[k * k]
 * output or NULL.  Each group is then one consensus problem; solve them
 * together with mcc_consensus_batch. */
int mcc_group_partitions(const int32_t* const* labels, int32_t k, int64_t n, int64_t lambda,
                         int32_t* group, int32_t* ngroups, int64_t* lambda_used, int64_t* dist,
                         void* stream);

/* Free the workspace the library keeps between calls (every device and
 * stream), and the batched launch's graphs.  Call it with no other libmcc
 * call in flight.  Returns 0 or MCC_EDEVICE. */
int mcc_release_workspace(void);

/* Static text for a return code (for MCC_EDEVICE, the last HIP error seen
 * on this thread). */
const char* mcc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
