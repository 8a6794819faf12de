// Internal declarations shared by the kernels and the host driver of libmcc.
// Not part of the public interface (include/mcc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcc {

constexpr int kBlock = 256;  // threads per workgroup for every kernel here

// Device-resident control block of one solve.  The pass loop is driven from
// the device: every kernel of a pass reads `done` first and returns at once
// when the solve has finished, so the host can enqueue several passes
// without waiting for each.
struct Ctl {
  int32_t done;             // 1 once no further pass may run
  int32_t fallback;         // 1 if the current pass commits only a subset
  int32_t nprop;            // proposals of the current pass
  int32_t committed;        // moves committed by the current fallback pass
  int32_t passes;           // scoring passes run
  int32_t converged;        // 1 when a pass finds no proposal
  int32_t fallback_rounds;  // passes that fell back
  int32_t max_rounds;       // pass cap
  int32_t k;                // number of input partitions
  int32_t err;              // input error bits (see kErr*)
  int64_t pass_evals;       // candidate clusters scored in the current pass
  int64_t evals;            // candidate clusters scored in all passes
  int64_t dS2;              // change of sum_c s_c^2 caused by tracked updates
  int64_t dN2;              // change of sum_i sum_(c,l) N_i(c,l)^2, same
  int64_t O;                // current objective sum_i Mirkin(C, P_i)
  int64_t moves;            // committed moves in all passes
  int64_t boundary;         // vertices with a candidate, summed over passes
  int32_t heavy_count;      // vertices deferred by the tiled scorer this pass
  int32_t rescore_count;    // vertices the status kernel left for scoring
  int32_t plist_count;      // proposers of the current pass (k_props)
  int32_t defer_all;        // 1: this pass's vertices all go to the wave-per-vertex
                            // scorer (most had too many candidates for the tiles)
  int64_t skipped;          // candidate evaluations proven unnecessary (all passes)
  int64_t prop_rows;        // hashed rows: rows the current pass's proposals can add
  int64_t* trace;           // device int64[max_rounds * 4] or null
};

constexpr int32_t kErrNegLabel = 1;
constexpr int32_t kErrInitRange = 2;
constexpr int32_t kErrGraph = 4;

// Contingency tables N_i(x, l): the number of vertices of consensus cluster
// x (dense index) whose label id in partition i is l.  Three layouts:
//  - blocked:     N[toff[i] + x * L[i] + l], one dense block per partition;
//  - interleaved: N[(x * Lmax + l) * k + i], the k partitions of one
//    (cluster, label id) pair side by side.  With label ids aligned to the
//    consensus cluster each label mostly overlaps (any injective relabelling
//    leaves every count unchanged), the k probes of one vertex and cluster
//    mostly fall into one cache line;
//  - hashed: one open-addressing table (linear probing) of 16-byte slots
//    {uint64 key, int32 count, unused}, key = x << 32 | (toff[i] + l) with
//    toff[i] the first global label id of partition i, for cluster counts
//    whose dense tables would not fit (e.g. singleton starts).  Keys are
//    never removed; a slot whose count drops to 0 stays, and the table is
//    rebuilt from the partition before it could fill beyond half;
//  - hashed rows: the same open addressing over keys x << 32 | l alone
//    (rkeys, 8 bytes a row), each key owning a row of k counts N[r * k + i]
//    (partition i, label id l in that partition).  With the label ids of
//    every partition aligned to one reference partition, most partitions
//    give a vertex the same id, so the k counts a vertex reads for one
//    cluster mostly share one key and one row.
// A "cell" is the index of one counter: the dense position, or the slot.
struct Tables {
  int32_t* N;           // dense: the counts; hashed: the slots as int32 words
  const int64_t* toff;  // blocked: start of partition i; hashed: label id offset
  const int32_t* L;     // ids of partition i lie in [0, L[i])
  int32_t Lmax;         // interleaved: ids of every partition lie in [0, Lmax)
  int32_t k;
  int32_t interleaved;
  int32_t hashed;
  int32_t hshift;       // hashed: 64 - log2(slots)
  int32_t pad;
  uint64_t hmask;       // hashed: slots - 1
  int32_t* hocc;        // hashed: occupied slots
  int32_t* herr;        // hashed: set if an insert found no slot
  uint64_t* rkeys;      // hashed rows: the row keys (N holds the rows' counts)
  int32_t rows;         // 1: hashed rows
  int32_t pad2;
};

constexpr uint64_t kHashEmpty = ~0ull;

// Dense cell of (partition i, cluster x, label id l).  Every table holds
// fewer than 2^31 cells (checked when it is sized), so the index is
// computed in 32 bits.
__device__ inline uint32_t cell(const Tables& t, int i, int32_t x, int32_t l) {
  return t.interleaved ? ((uint32_t)x * (uint32_t)t.Lmax + (uint32_t)l) * (uint32_t)t.k + i
                       : (uint32_t)t.toff[i] + (uint32_t)x * (uint32_t)t.L[i] + (uint32_t)l;
}

__device__ inline uint64_t hkey(const Tables& t, int i, int32_t x, int32_t l) {
  return t.rows ? (((uint64_t)(uint32_t)x << 32) | (uint64_t)(uint32_t)l)
                : (((uint64_t)(uint32_t)x << 32) | (uint64_t)(t.toff[i] + l));
}

__device__ inline uint64_t hstart(const Tables& t, uint64_t key) {
  return (key * 0x9E3779B97F4A7C15ull) >> t.hshift;  // Fibonacci hashing
}

// Count stored under `key`, 0 if absent (reads only: the table is frozen).
__device__ inline int32_t hget(const Tables& t, uint64_t key) {
  const uint4* H = reinterpret_cast<const uint4*>(t.N);
  uint64_t h = hstart(t, key);
  for (uint64_t q = 0; q <= t.hmask; ++q) {
    const uint4 e = H[h];
    const uint64_t kk = ((uint64_t)e.y << 32) | e.x;
    if (kk == key) return (int32_t)e.z;
    if (kk == kHashEmpty) return 0;
    h = (h + 1) & t.hmask;
  }
  return 0;
}

// Slot of `key`, claimed if absent (then `claimed` is incremented: callers
// add their claims to *hocc once per wave, flush_claims).  The table is
// sized and rebuilt so that it is never more than half full; should no slot
// be found, *herr is set (the solve then reports an error) and slot 0 is
// returned.
__device__ inline uint32_t hslot(const Tables& t, uint64_t key, int32_t& claimed) {
  unsigned long long* H = reinterpret_cast<unsigned long long*>(t.N);
  uint64_t h = hstart(t, key);
  for (uint64_t q = 0; q <= t.hmask; ++q) {
    const uint64_t kk = H[2 * h];
    if (kk == key) return (uint32_t)h;
    if (kk == kHashEmpty) {
      const uint64_t prev = atomicCAS(&H[2 * h], (unsigned long long)kHashEmpty,
                                      (unsigned long long)key);
      if (prev == kHashEmpty) {
        ++claimed;
        return (uint32_t)h;
      }
      if (prev == key) return (uint32_t)h;
    }
    h = (h + 1) & t.hmask;
  }
  atomicOr(t.herr, 1);
  return 0;
}

// Hashed rows: the row of `key`, -1 if absent (reads only).
__device__ inline int64_t rfind(const Tables& t, uint64_t key) {
  uint64_t h = hstart(t, key);
  for (uint64_t q = 0; q <= t.hmask; ++q) {
    const uint64_t kk = t.rkeys[h];
    if (kk == key) return (int64_t)h;
    if (kk == kHashEmpty) return -1;
    h = (h + 1) & t.hmask;
  }
  return -1;
}

// Hashed rows: the row of `key`, claimed if absent (as hslot).
__device__ inline uint32_t rslot(const Tables& t, uint64_t key, int32_t& claimed) {
  unsigned long long* K = reinterpret_cast<unsigned long long*>(t.rkeys);
  uint64_t h = hstart(t, key);
  for (uint64_t q = 0; q <= t.hmask; ++q) {
    const uint64_t kk = K[h];
    if (kk == key) return (uint32_t)h;
    if (kk == kHashEmpty) {
      const uint64_t prev = atomicCAS(&K[h], (unsigned long long)kHashEmpty,
                                      (unsigned long long)key);
      if (prev == kHashEmpty) {
        ++claimed;
        return (uint32_t)h;
      }
      if (prev == key) return (uint32_t)h;
    }
    h = (h + 1) & t.hmask;
  }
  atomicOr(t.herr, 1);
  return 0;
}

// The counter of a cell (hashed rows: cells are row * k + i).
__device__ inline int32_t* counter(const Tables& t, uint32_t c) {
  return (t.hashed && !t.rows) ? t.N + 4 * (uint64_t)c + 2 : t.N + c;
}

// Cell of (i, x, l) for an update: the dense position, or the key's slot
// (claimed if new), or its row's counter of partition i.
__device__ inline uint32_t cell_upd(const Tables& t, int i, int32_t x, int32_t l,
                                    int32_t& claimed) {
  if (!t.hashed) return cell(t, i, x, l);
  if (t.rows) return rslot(t, hkey(t, i, x, l), claimed) * (uint32_t)t.k + (uint32_t)i;
  return hslot(t, hkey(t, i, x, l), claimed);
}

// Hashed tables: the count of (i, x, l), 0 if absent.
__device__ inline int32_t hcount(const Tables& t, int i, int32_t x, int32_t l) {
  if (t.rows) {
    const int64_t r = rfind(t, hkey(t, i, x, l));
    return r < 0 ? 0 : t.N[(uint64_t)r * (uint64_t)t.k + (uint64_t)i];
  }
  return hget(t, hkey(t, i, x, l));
}

// Hashed rows: N[row(C[v], Lvm[j]) k + i] += 1 for every j = v k + i in
// [0, n k), the grid's threads (tid of stride) taking four items at a time
// with their first probes in flight together (a key found there needs no
// probe loop).  The wave's claims are added to the occupancy counter.
__device__ inline int32_t rows_count(const Tables& t, const int32_t* __restrict__ C,
                                     const int32_t* __restrict__ Lvm, int64_t n, int32_t k,
                                     int64_t tid, int64_t stride) {
  constexpr int U = 4;
  int32_t claimed = 0;
  const int64_t total = n * k;
  for (int64_t j0 = tid; j0 < total; j0 += U * stride) {
    uint64_t key[U], h[U], kk[U];
    int32_t ii[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * stride;
      ok[u] = j < total;
      const int64_t jc = ok[u] ? j : 0;
      const int64_t v = jc / k;
      ii[u] = (int32_t)(jc - v * k);
      key[u] = hkey(t, 0, C[v], Lvm[jc]);
      h[u] = hstart(t, key[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) kk[u] = t.rkeys[h[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const uint64_t r = kk[u] == key[u] ? h[u] : (uint64_t)rslot(t, key[u], claimed);
      atomicAdd(t.N + r * (uint64_t)t.k + (uint64_t)ii[u], 1);
    }
  }
  return claimed;
}

// Add the wave's claimed slots to the occupancy counter (all lanes of the
// wave call it).
__device__ inline void flush_claims(const Tables& t, int32_t claimed) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) claimed += __shfl_xor(claimed, o, 64);
  if ((threadIdx.x & 63) == 0 && claimed) atomicAdd(t.hocc, claimed);
}

// Count of (i, x, l) for scoring.
__device__ inline int32_t count_of(const Tables& t, int i, int32_t x, int32_t l) {
  return t.hashed ? hcount(t, i, x, l) : t.N[cell(t, i, x, l)];
}

// ---- setup kernels (setup.hip) -------------------------------------------
void launch_label_max(const int32_t* const* dlabels, int32_t k, int64_t n, int32_t* maxlab,
                      int32_t* err, hipStream_t st);
void launch_label_mark(const int32_t* const* dlabels, int32_t k, int64_t n,
                       const int64_t* loff, int32_t* flags, hipStream_t st);
void launch_scan(const int32_t* in, int32_t* out, int64_t len, int32_t* tmp, hipStream_t st);
int64_t scan_tmp_elems(int64_t len);
void launch_label_counts(const int32_t* scan, const int64_t* loff, int32_t k, int32_t* Lc,
                         hipStream_t st);
// fmap[loff[i] + x] = dense id of raw label x of partition i (where present)
void launch_label_ids(const int32_t* scan, const int64_t* loff, int32_t k, int64_t max_span,
                      int32_t* fmap, hipStream_t st);
void launch_label_transpose(const int32_t* const* dlabels, int32_t k, int64_t n,
                            const int64_t* loff, const int32_t* fmap, int32_t* Lvm,
                            hipStream_t st);
// Label alignment from a blocked table: amap[poff[i] + l] = new id of dense
// label l of partition i, L2[i] = new id bound of partition i.
void launch_align(const Tables& blocked, int32_t k, int32_t K0, int32_t maxL,
                  const int64_t* poff, int64_t total_labels, uint64_t* win, int32_t* home,
                  uint64_t* key, int32_t* extra, int32_t* rank, int32_t* scan_tmp,
                  int32_t* amap, int32_t* L2, hipStream_t st);
void launch_fmap_update(const int32_t* scan, const int64_t* loff, const int64_t* poff,
                        const int32_t* amap, int32_t k, int64_t max_span, int32_t* fmap,
                        hipStream_t st);
void launch_cluster_mark(const int32_t* init, int64_t n, int32_t* flags, int32_t* err,
                         hipStream_t st);
void launch_cluster_assign(const int32_t* init, int64_t n, const int32_t* cmap, int32_t* C,
                           int32_t* rawid, hipStream_t st);
void launch_iota(int32_t* a, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st);
void launch_fill_u64(uint64_t* a, int64_t n, uint64_t v, hipStream_t st);
// Counts a sample of the vertices, runs of 64 consecutive vertices one run
// in every `stride` (stride 1: all vertices, the exact tables).
// max_l: the largest label id bound of the table's partitions.
void launch_build(const int32_t* C, const int32_t* const* dlabels, const int64_t* loff,
                  const int32_t* fmap, int64_t n, int32_t k, int32_t K0, int32_t max_l, Tables t,
                  hipStream_t st, int64_t stride = 1);
void launch_sizes(const int32_t* C, int64_t n, int32_t K0, int32_t* s, hipStream_t st);
// Label sizes |P_i l| counted from the labels: the ids label l of
// partition i has in some layout (labels[i][v] through fmap + loff[i]) lie
// in [0, lpoff[i + 1] - lpoff[i]); hist (lpoff[k] entries) is scratch.
struct LabelHist {
  const int32_t* const* dlabels;
  const int64_t* loff;
  const int32_t* fmap;
  const int64_t* lpoff;
  int64_t total_labels;
  int32_t* hist;
};
// acc[0] += sum_x s_x^2; acc[1] += sum_i sum_l |P_i l|^2 (summed over the
// table's cells when it has at most n k of them, else from the label
// histogram); acc[2] += sum over cells of N^2: a scan of the `total_entries`
// cells, or, when the label rows Lvm are given and the table is much larger
// than n k, the sum over vertices and partitions of N_i(C(v), l_i(v)).
// maxL: the largest label id bound of the table's partitions.
void launch_objective0(const Tables& t, int32_t k, int32_t K0, int32_t maxL, const int32_t* s,
                       int64_t total_entries, const LabelHist& lh, const int32_t* C,
                       const int32_t* Lvm, int64_t n,
                       int64_t* acc /* 3 int64: sum s^2, sum hist^2, sum N^2 */,
                       hipStream_t st);
// Hashed tables: empty every slot; the objective from label histograms
// (hist: int32[total_labels] scratch) and the slot counts.
void launch_hash_clear(Tables t, hipStream_t st);
// singletons (K0 = n): every cell holds 0 or 1, so sum N^2 = n k without a scan.
void launch_objective0_hashed(const Tables& t, const int32_t* const* dlabels, const int64_t* loff,
                              const int32_t* fmap, int64_t n, int32_t k, int32_t K0,
                              const int32_t* s, int64_t total_labels, int32_t* hist,
                              bool singletons, int64_t* acc, hipStream_t st);
// Hashed rows: the reference labels (partition 0's label ids) the other
// partitions are aligned to, and each vertex's distinct label ids (the
// rows it contributes to; *total, zeroed by the caller, gets their sum).
void launch_ref_labels(const int32_t* const* dlabels, const int64_t* loff, const int32_t* fmap,
                       int64_t n, int32_t* Cref, hipStream_t st);
void launch_row_distinct(const int32_t* Lvm, int64_t n, int32_t k, uint8_t* rdist, int64_t* total,
                         hipStream_t st);
// Hashed rows: the counts of C from the vertex-major label rows.
void launch_build_rows(const int32_t* C, const int32_t* Lvm, int64_t n, int32_t k, Tables t,
                       hipStream_t st);
// In-arc lists: in_ptr (exclusive scan of in-degrees, n + 1) and in_pos
// (arc positions grouped by head vertex); ac[j] = C[col[j]].
void launch_in_degree(const int32_t* col, int64_t nnz, int32_t* indeg, hipStream_t st);
void launch_in_fill(const int32_t* col, int64_t nnz, int32_t* cursor, int32_t* in_pos,
                    hipStream_t st);
void launch_arc_clusters(const int32_t* col, int64_t nnz, const int32_t* C, int32_t* ac,
                         hipStream_t st);
void launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t st);
void launch_narrow(const int32_t* src, void* dst, int32_t bytes, int64_t n, hipStream_t st);
void launch_validate_csr(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* err, hipStream_t st);
// err |= kErrGraph unless every arc (v, u) has a reverse arc (u, v).
void launch_check_symmetric(const int64_t* row_ptr, const int32_t* col, int64_t n,
                            int32_t* err, hipStream_t st);
void launch_finish(const int32_t* C, const int32_t* rawid, int64_t n, int32_t* out,
                   hipStream_t st);
void launch_count_nonzero(const int32_t* a, int64_t n, int32_t* count, hipStream_t st);
void launch_first_occurrence(const int32_t* in, int64_t n, int32_t* first, hipStream_t st);
void launch_first_flags(const int32_t* in, int64_t n, const int32_t* first, int32_t* flags,
                        hipStream_t st);
void launch_canonical_write(const int32_t* in, int64_t n, const int32_t* first,
                            const int32_t* rank, int32_t* out, hipStream_t st);

// ---- comparison kernels (metrics.hip) --------------------------------------
int cell_stats_blocks(int64_t cells);
int xlogx_blocks(int64_t len);
// Over the cells of a one-partition table: row/column maxima and column sums
// (rowmax, colmax, colsum zeroed by the caller), per-block sums of c ln c.
void launch_cell_stats(const Tables& t, int64_t cells, int32_t Lb, int32_t* rowmax,
                       int32_t* colmax, int32_t* colsum, double* partial, hipStream_t st);
void launch_xlogx(const int32_t* a, int64_t len, double* partial, hipStream_t st);
void launch_sum_partials(const double* partial, int32_t count, double* out, hipStream_t st);
void launch_sum_i32(const int32_t* a, int64_t len, int64_t* acc, hipStream_t st);
// Split-join distance of npairs partition pairs (T zeroed by the caller,
// poff[p] its cells for pair p).
void launch_pair_tables(const int32_t* D, int64_t n, const int32_t* pi, const int32_t* pj,
                        const int64_t* poff, const int32_t* L, int32_t npairs, int32_t* T,
                        hipStream_t st);
void launch_pair_split_join(const int32_t* T, const int32_t* pi, const int32_t* pj,
                            const int64_t* poff, const int32_t* L, int32_t npairs, int64_t n,
                            int64_t* dist, hipStream_t st);

// ---- pass kernels (pass.hip) ----------------------------------------------
struct PassArgs {
  Ctl* ctl;
  int64_t n;
  int32_t k;
  int32_t literal;
  const int64_t* row_ptr;
  const int32_t* col;
  int32_t* C;
  const int32_t* Lvm;
  Tables t;
  int32_t* s;
  int32_t* prop;      // proposed target cluster, -1 none; fallback marks
  int64_t* dprop;     // gain of the proposal
  uint64_t* owner;    // per cluster, fallback owners
  int32_t* heavy;     // [n] vertices the tiled scorer defers to the group scorer
  // ac[j] = C[col[j]]: the cluster at the head of every arc, kept current by
  // rewriting the in-arcs of each vertex that moves (in_pos[in_ptr[u] ..
  // in_ptr[u + 1]) are the arcs pointing at u), so that scoring streams
  // arcs instead of gathering clusters
  int32_t* ac;
  const int32_t* in_ptr;
  const int32_t* in_pos;
  int64_t cells;      // table cells (keys >= cells address cluster sizes)
  int32_t* hflag;     // hashed tables: 1 while the current pass rebuilds them
  const uint8_t* rdist;  // hashed rows: distinct label ids of each vertex (the rows
                         // its move can add), else null
  // Hashed tables: member lists of the clusters as they stand at the start of
  // the pass (members[mstart[x] .. mstart[x + 1]) are the vertices of x), so
  // that a small cluster's agreement sum is taken over its members' label
  // rows instead of k table probes.  Null otherwise.
  int32_t* mstart;    // K0 + 1
  int32_t* mcnt;      // K0 (fill cursors)
  int32_t* members;   // n
  int32_t* mscan_tmp;
  int32_t msum_max;   // largest cluster scored from member rows (at most
                      // kMemberSumMax): a member row costs two or three
                      // lines, a key table's probes k lines, a row table's
                      // a few
  int32_t K0;
  // Narrow copy of C (uint8 when K0 <= 256, uint16 when K0 <= 65536, else
  // C itself) for the per-arc cluster gathers: a few MiB stay resident in
  // every XCD's L2 where the int32 array would not.
  void* Cn;
  int32_t cn_bytes;
  int32_t arcs_aligned;  // col (and ac) start on a 16-byte boundary
  int64_t nnz;
  // Symmetric graphs (every arc has its reverse): candidate sets carried
  // over between passes.  A vertex is dirty when it or a neighbour moved in
  // the previous pass (a move marks the mover and its out-neighbours, which
  // are its in-neighbours); a clean vertex with a cached set (cnum >= 0)
  // skips its arcs.  Null when off.
  int32_t* dirty;     // n
  int32_t* cnum;      // n: cached candidate count, -1 none
  int32_t* ccache;    // n * kCacheCand
  // Skipping provably unchanged decisions (with the candidate cache).  The
  // gain of v for x, 2 (S_c(v) - S_x(v)) + k (|x| - |c| - 1), moves by at
  // most k for every vertex that enters or leaves c or x (each changes
  // 2 S_y(v) - k |y| by 2 agree(u, v) - k, between -k and k).  slack[v] is
  // the smallest gain of v at its last exact scoring (clamped to int32, -1:
  // none or negative) minus the bounds of the passes since; churn counts the
  // vertices that entered or left each cluster in the previous pass
  // (churn[(p & 1) K0 ..] is read by pass p; the other half is filled by
  // its apply).  A clean vertex whose slack stays >= 0 after subtracting
  // k (churn of its cluster + largest churn of its cached candidates)
  // cannot propose, and is not rescored.
  int32_t* slack;     // n
  int32_t* churn;     // 2 * K0
  // Per-pass status (with the candidate cache), written by k_status:
  // st[v] = -1 when v is settled for this pass (no candidate, or skipped by
  // the bound; its proposal is already written), 0 when its candidates must
  // be found from its arcs, c > 0 when its c cached candidates must be
  // rescored.  rlist holds the vertices with st >= 0 (rescore_count of
  // them).  Passes with more than sparse_max of them run the tiled scorer
  // over all tiles, the others the list scorer over rlist.
  int32_t* st;        // n
  int32_t* rlist;     // n
  int32_t sparse_max;
  int32_t pad3;
  // Per-pass counters of the scoring kernels (kPassCounters of them, each in
  // its own 512-byte line so that their atomics do not share an L2 channel),
  // added once per workgroup and folded into the control block by k_begin.
  int64_t* pc;        // kPassCounters * kCounterStride
  // The proposers of the pass, listed by k_props: the batch apply then runs
  // on as many workgroups as the proposals need, so that a counter that many
  // proposals update receives one atomic from each of few workgroups.
  int32_t* plist;     // n
  // Dense tables whose per-partition slice (K0 x label ids) plus two K0
  // arrays fit kDeltaLdsMax bytes of LDS use the histogram apply
  // (k_apply_delta) with that much dynamic LDS and delta_slices slices of
  // the proposal list; 0: the hashed aggregation (k_apply_all).
  int32_t delta_lds;
  int32_t delta_slices;
};

constexpr int kDeltaLdsMax = 48 << 10;

constexpr int kPassCounters = 5;    // evaluations, proposals, boundary vertices, skipped,
                                    // boundary vertices with more candidates than a tile holds
constexpr int kCounterStride = 64;  // int64 words between two counters

constexpr int kCacheCand = 8;  // candidate clusters cached per vertex

// Compile-time variants: CN is the narrow copy's width in bytes (0: read the
// per-arc cache), IL selects the interleaved table layout.
template <int CN>
__device__ inline int32_t cn_load_t(const PassArgs& a, int64_t j, int32_t u) {
  if (CN == 0) return a.ac[j];
  if (CN == 1) return ((const uint8_t*)a.Cn)[u];
  if (CN == 2) return ((const uint16_t*)a.Cn)[u];
  return ((const int32_t*)a.Cn)[u];
}

// Largest cluster whose agreement sum is taken over its members' label rows
// when the table is hashed: s rows of 4k bytes streamed against k random
// probes of a table in HBM.
constexpr int32_t kMemberSumMax = 16;

// Table layouts as compile-time variants.
enum TableKind { kBlocked = 0, kInterleaved = 1, kHashed = 2 };

template <int TK>
__device__ inline int32_t count_t(const Tables& t, int i, int32_t x, int32_t l) {
  if (TK == kInterleaved)
    return t.N[((uint32_t)x * (uint32_t)t.Lmax + (uint32_t)l) * (uint32_t)t.k + i];
  if (TK == kHashed) return hcount(t, i, x, l);
  return t.N[(uint32_t)t.toff[i] + (uint32_t)x * (uint32_t)t.L[i] + (uint32_t)l];
}

__device__ inline int32_t cn_load(const PassArgs& a, int64_t u) {
  if (a.cn_bytes == 1) return ((const uint8_t*)a.Cn)[u];
  if (a.cn_bytes == 2) return ((const uint16_t*)a.Cn)[u];
  return ((const int32_t*)a.Cn)[u];
}

__device__ inline void cn_store(const PassArgs& a, int64_t u, int32_t c) {
  if (a.cn_bytes == 1) ((uint8_t*)a.Cn)[u] = (uint8_t)c;
  else if (a.cn_bytes == 2) ((uint16_t*)a.Cn)[u] = (uint16_t)c;
  else ((int32_t*)a.Cn)[u] = c;
}

// Exclusive scan of one value per thread over a kBlock-thread workgroup;
// *total receives the sum.  Contains barriers: call from all threads.
__device__ inline int32_t block_exclusive_scan(int32_t x, int32_t* total) {
  __shared__ int32_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t v = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int32_t off = 0, tot = 0;
#pragma unroll
  for (int j = 0; j < kBlock / 64; ++j) {
    if (j < w) off += wsum[j];
    tot += wsum[j];
  }
  __syncthreads();
  *total = tot;
  return off + v - x;
}

// lanes 0: tiled scorer (with the group scorer for deferred vertices);
// 4..64: group scorer with that many lanes per vertex.
bool score_lanes_ok(int lanes);
// Enqueue one pass; when the events are given they bracket the scoring
// kernel on the same stream.
void enqueue_pass(const PassArgs& a, int lanes, int grid_score, int grid_apply, hipStream_t st,
                  hipEvent_t score_begin = nullptr, hipEvent_t score_end = nullptr);
void launch_ctl_init(Ctl* ctl, const int64_t* acc, int32_t k, int32_t max_rounds,
                     int64_t* trace, hipStream_t st);

}  // namespace mcc
