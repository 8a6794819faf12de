// Setup kernels of libmcc: label compaction and transpose, consensus-cluster
// compaction, contingency-table build, objective reduction, CSR validation
// and presentation relabelling.
//
// The contingency counts N_i(x, l) (members of consensus cluster x put in
// cluster l by input partition i) and cluster sizes s_x are what the
// closed-form gain of a move needs; the paper instead sums over cluster
// members (Methods, "Computation and memory complexity"), which costs
// O(|cluster| k) per candidate where these tables cost O(k).
#include <algorithm>

#include "impl.h"

namespace mcc {

namespace {

inline int grid_for(int64_t items, int per_block, int cap = 65535) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

template <typename T>
__device__ T block_sum(T x) {
  __shared__ T part[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  T t = 0;
  if (threadIdx.x == 0)
    for (int j = 0; j < kBlock / 64; ++j) t += part[j];
  __syncthreads();
  return t;  // valid in thread 0
}

// ---- scan ------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t* __restrict__ in,
                                                        int64_t len, int32_t* __restrict__ tmp) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    int64_t idx = base + (int64_t)j * kBlock + threadIdx.x;
    if (idx < len) s += in[idx];
  }
  int32_t t = block_sum<int32_t>(s);
  if (threadIdx.x == 0) tmp[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_scan_top(int32_t* __restrict__ tmp, int64_t nb) {
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    int64_t idx = b0 + threadIdx.x;
    int32_t x = idx < nb ? tmp[idx] : 0;
    int32_t tot;
    int32_t e = block_exclusive_scan(x, &tot);
    if (idx < nb) tmp[idx] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) tmp[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int32_t* __restrict__ in, int64_t len,
                                                      const int32_t* __restrict__ tmp,
                                                      int32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t vals[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t idx = base + j;
    vals[j] = idx < len ? in[idx] : 0;
    s += vals[j];
  }
  int32_t tot;
  int32_t run = tmp[blockIdx.x] + block_exclusive_scan(s, &tot);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t idx = base + j;
    if (idx < len) out[idx] = run;
    run += vals[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[len] = tmp[gridDim.x];
}

// ---- labels ----------------------------------------------------------------
// Visits the labels p[0, n) of one partition, spread over the x dimension
// of the grid: 16-byte loads over the aligned middle of the row, four of them
// in flight per thread and handed to f16 as sixteen labels, single loads
// for the unaligned head and the tail, handed to f.  Past the end of the
// middle, loads are clamped to its last word instead of branched around, so
// a label may be visited more than once: f and f16 must be idempotent.
// Label rows are seen as global memory: their loads are global, not flat,
// so that waits on scalar and LDS operations do not wait on them too.
typedef __attribute__((address_space(1))) int32_t global_i32;
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) i32x4 global_i4;

template <typename F, typename F16>
__device__ inline void for_each_label(const int32_t* __restrict__ row, int64_t n, F&& f,
                                      F16&& f16) {
  const global_i32* __restrict__ p = (const global_i32*)row;
  const int64_t head = min(n, (int64_t)(((16 - ((uintptr_t)p & 15)) & 15) >> 2));
  const int64_t nv = (n - head) >> 2;  // 16-byte words
  const int64_t tail = head + nv * 4;
  const int64_t t = gtid(), T = gstride();
  if (t < head) f(p[t]);
  if (t < n - tail) f(p[tail + t]);
  const global_i4* __restrict__ q = (const global_i4*)(p + head);
  for (int64_t w = t; w < nv; w += 4 * T) {
    const i32x4 a = q[w], b = q[min(w + T, nv - 1)], c = q[min(w + 2 * T, nv - 1)],
                d = q[min(w + 3 * T, nv - 1)];
    const int32_t x[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w,
                           c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
    f16(x);
  }
}

__global__ __launch_bounds__(kBlock) void k_label_max(const int32_t* const* __restrict__ labels,
                                                      int64_t n, int32_t* __restrict__ maxlab,
                                                      int32_t* __restrict__ err) {
  __shared__ int32_t s_m[kBlock / 64], s_lo[kBlock / 64];
  int32_t m = -1, lo = 0;
  auto f = [&](int32_t x) {
    m = max(m, x);
    lo = min(lo, x);
  };
  for_each_label(labels[blockIdx.y], n, f, [&](const int32_t(&x)[16]) {
#pragma unroll
    for (int j = 0; j < 16; ++j) f(x[j]);
  });
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = max(m, __shfl_xor(m, o, 64));
    lo = min(lo, __shfl_xor(lo, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    s_m[threadIdx.x >> 6] = m;
    s_lo[threadIdx.x >> 6] = lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per workgroup
    for (int j = 1; j < kBlock / 64; ++j) {
      m = max(m, s_m[j]);
      lo = min(lo, s_lo[j]);
    }
    atomicMax(&maxlab[blockIdx.y], m);
    if (lo < 0) atomicOr(err, kErrNegLabel);
  }
}

__global__ __launch_bounds__(kBlock) void k_label_mark(const int32_t* const* __restrict__ labels,
                                                       int64_t n, const int64_t* __restrict__ loff,
                                                       int32_t* __restrict__ flags) {
  int32_t* f = flags + loff[blockIdx.y];
  // most labels repeat: skip the store when the flag is set; sixteen flags
  // are read before any is written (a label seen twice is written twice)
  for_each_label(
      labels[blockIdx.y], n, [&](int32_t x) { if (!f[x]) f[x] = 1; },
      [&](const int32_t(&x)[16]) {
        int32_t seen[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) seen[j] = f[x[j]];
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (!seen[j]) f[x[j]] = 1;
      });
}

__global__ void k_label_counts(const int32_t* __restrict__ scan, const int64_t* __restrict__ loff,
                               int32_t k, int32_t* __restrict__ Lc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) Lc[i] = scan[loff[i + 1]] - scan[loff[i]];
}

// fmap[loff[i] + x] = dense id of label x of partition i, for present labels
__global__ __launch_bounds__(kBlock) void k_label_ids(const int32_t* __restrict__ scan,
                                                      const int64_t* __restrict__ loff,
                                                      int32_t* __restrict__ fmap) {
  const int i = blockIdx.y;
  const int64_t b = loff[i], e = loff[i + 1];
  const int32_t base = scan[b];
  for (int64_t p = b + gtid(); p < e; p += gstride()) fmap[p] = scan[p] - base;
}

// Relabel present labels through the alignment map.
__global__ __launch_bounds__(kBlock) void k_fmap_update(const int32_t* __restrict__ scan,
                                                        const int64_t* __restrict__ loff,
                                                        const int64_t* __restrict__ poff,
                                                        const int32_t* __restrict__ amap,
                                                        int32_t* __restrict__ fmap) {
  const int i = blockIdx.y;
  const int64_t b = loff[i], e = loff[i + 1];
  const int32_t* am = amap + poff[i];
  for (int64_t p = b + gtid(); p < e; p += gstride())
    if (scan[p + 1] > scan[p]) fmap[p] = am[fmap[p]];
}

// Label ids, transposed to vertex-major rows: Lvm[v * k + i] = id of
// P_i(v).  A workgroup moves a tile of tv vertices x k partitions through
// LDS: waves read 64-vertex pieces of partition rows (eight pieces in flight
// per wave), then the workgroup writes the tile's rows * k outputs, which are
// contiguous, in order.
__global__ __launch_bounds__(kBlock) void k_label_transpose(
    const int32_t* const* __restrict__ labels, int32_t k, int64_t n,
    const int64_t* __restrict__ loff, const int32_t* __restrict__ fmap, int tv,
    int32_t* __restrict__ Lvm) {
  extern __shared__ int32_t tile[];  // [k][tv + 1], then one spare word
  constexpr int kWaves = kBlock / 64, kInFlight = 8;
  const int64_t v0 = (int64_t)blockIdx.x * tv;
  const int rows = (int)min((int64_t)tv, n - v0);
  // the wave index through a scalar register, so that the partition of a
  // piece, its row pointer and its label map offset are scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cpr = (rows + 63) >> 6;  // 64-vertex pieces per partition row
  const int items = k * cpr;
  for (int b = wave; b < items; b += kInFlight * kWaves) {
    // indexes clamped into the tile instead of branches, so that all the
    // loads issue before the first wait (a clamped lane reloads a valid
    // label and drops it)
    int32_t x[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int it = min(b + u * kWaves, items - 1), i = it / cpr;
      const global_i32* row = (const global_i32*)labels[i];
      x[u] = row[v0 + min((it - i * cpr) * 64 + lane, rows - 1)];
    }
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int it = min(b + u * kWaves, items - 1), i = it / cpr;
      x[u] = fmap[loff[i] + x[u]];
    }
    // a clamped lane writes the spare word past the tile
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) {
      const int it0 = b + u * kWaves, it = min(it0, items - 1), i = it / cpr;
      const int vv = (it - i * cpr) * 64 + lane;
      tile[it0 < items && vv < rows ? i * (tv + 1) + vv : k * (tv + 1)] = x[u];
    }
  }
  __syncthreads();
  int32_t* dst = Lvm + v0 * k;
  const int total = rows * k, sv = kBlock / k, si = kBlock - sv * k;
  int vv = threadIdx.x / k, i = threadIdx.x - vv * k;
  for (int f = threadIdx.x; f < total; f += kBlock) {
    dst[f] = tile[i * (tv + 1) + vv];
    i += si;
    vv += sv;
    if (i >= k) {
      i -= k;
      ++vv;
    }
  }
}

// The same for a partition count too large for a useful LDS tile: each
// thread writes one output, reading its label directly.
__global__ __launch_bounds__(kBlock) void k_label_transpose_direct(
    const int32_t* const* __restrict__ labels, int32_t k, int64_t n,
    const int64_t* __restrict__ loff, const int32_t* __restrict__ fmap,
    int32_t* __restrict__ Lvm) {
  for (int64_t f = gtid(); f < n * k; f += gstride()) {
    const int64_t v = f / k;
    const int32_t i = (int32_t)(f - v * k);
    Lvm[f] = fmap[loff[i] + labels[i][v]];
  }
}

// ---- consensus clusters ----------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_cluster_mark(const int32_t* __restrict__ init, int64_t n,
                                                         int32_t* __restrict__ flags,
                                                         int32_t* __restrict__ err) {
  int bad = 0;
  for (int64_t v = gtid(); v < n; v += gstride()) {
    int32_t x = init[v];
    if (x < 0 || x >= n) bad = 1;
    else flags[x] = 1;
  }
  if (bad) atomicOr(err, kErrInitRange);
}

__global__ __launch_bounds__(kBlock) void k_cluster_assign(const int32_t* __restrict__ init,
                                                           int64_t n,
                                                           const int32_t* __restrict__ cmap,
                                                           int32_t* __restrict__ C,
                                                           int32_t* __restrict__ rawid) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    C[v] = cmap[init[v]];
    if (cmap[v + 1] > cmap[v]) rawid[cmap[v]] = (int32_t)v;
  }
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t* __restrict__ a, int64_t n) {
  for (int64_t v = gtid(); v < n; v += gstride()) a[v] = (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t x) {
  for (int64_t v = gtid(); v < n; v += gstride()) a[v] = x;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(uint64_t* __restrict__ a, int64_t n,
                                                     uint64_t x) {
  for (int64_t v = gtid(); v < n; v += gstride()) a[v] = x;
}

// ---- contingency tables ------------------------------------------------------
constexpr int kLdsHist = 16384;  // int32 entries privatised in LDS (64 KiB)
constexpr int64_t kSampleRun = 64;  // vertices per run of a sampled build

// Workgroup (b, i) counts the pairs (C(v), P_i(v)) of its vertex range for
// partition i.  When partition i's K0 x L[i] slice fits the LDS the launch
// sized (lds_cap entries, at most kLdsHist) the counts are gathered there and
// flushed once; otherwise they go straight to the global table.
__global__ __launch_bounds__(kBlock) void k_build(const int32_t* __restrict__ C,
                                                  const int32_t* const* __restrict__ labels,
                                                  const int64_t* __restrict__ loff,
                                                  const int32_t* __restrict__ fmap, int64_t n,
                                                  int32_t K0, Tables t, int64_t stride,
                                                  int32_t lds_cap) {
  extern __shared__ int32_t h[];  // lds_cap entries, sized by the launch
  const int i = blockIdx.y;
  const int32_t Li = t.L[i];
  const int64_t entries = (int64_t)K0 * Li;
  const bool lds = !t.hashed && entries > 0 && entries <= lds_cap;
  // Counts concentrate on few cells (a cluster's members mostly share their
  // labels), so threads spread over up to 8 copies of a small slice: fewer
  // atomics on one LDS word at a time.
  const int copies = lds ? (int)min((int64_t)8, lds_cap / max(entries, (int64_t)1)) : 1;
  int32_t* hc = h + (threadIdx.x % copies) * entries;
  if (lds) {
    for (int j = threadIdx.x; j < entries * copies; j += kBlock) h[j] = 0;
    __syncthreads();
  }
  // a sample of the vertices: runs of kSampleRun consecutive vertices, one
  // run every stride runs, so that the sample is read with whole cache
  // lines (stride 1: all vertices)
  const int64_t runs = (n + kSampleRun - 1) / kSampleRun;
  const int64_t ns = ((runs + stride - 1) / stride) * kSampleRun;
  const int64_t per = (ns + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = min(ns, j0 + per);
  // partition-major input labels (coalesced when stride is 1) mapped to their
  // ids, kBuildUnroll vertices a thread at a time: all their loads, then all
  // the label map gathers, then the counts (a lane past the end reloads
  // vertex 0 and counts nothing)
  const global_i32* p = (const global_i32*)labels[i];
  const int32_t* map = fmap + loff[i];
  int32_t claimed = 0;
  constexpr int kBuildUnroll = 8;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kBuildUnroll * kBlock) {
    int32_t x[kBuildUnroll], l[kBuildUnroll];
    bool ok[kBuildUnroll];
#pragma unroll
    for (int u = 0; u < kBuildUnroll; ++u) {
      const int64_t jj = j + u * kBlock;
      const int64_t v = (jj / kSampleRun) * (kSampleRun * stride) + jj % kSampleRun;
      ok[u] = jj < j1 && v < n;
      const int64_t vc = ok[u] ? v : 0;
      x[u] = C[vc];
      l[u] = p[vc];
    }
#pragma unroll
    for (int u = 0; u < kBuildUnroll; ++u) l[u] = map[l[u]];
#pragma unroll
    for (int u = 0; u < kBuildUnroll; ++u) {
      if (!ok[u]) continue;
      if (lds) atomicAdd(&hc[x[u] * Li + l[u]], 1);
      else atomicAdd(counter(t, cell_upd(t, i, x[u], l[u], claimed)), 1);
    }
  }
  if (t.hashed) flush_claims(t, claimed);
  if (lds) {
    __syncthreads();
    for (int j = threadIdx.x; j < entries; j += kBlock) {
      int32_t c = 0;
      for (int q = 0; q < copies; ++q) c += h[q * entries + j];
      if (c) {
        const int32_t x = j / Li;
        atomicAdd(&t.N[cell(t, i, x, j - x * Li)], c);
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sizes(const int32_t* __restrict__ C, int64_t n,
                                                  int32_t K0, int32_t* __restrict__ s) {
  __shared__ int32_t h[kLdsHist];
  const bool lds = K0 <= kLdsHist;
  if (lds) {
    for (int j = threadIdx.x; j < K0; j += kBlock) h[j] = 0;
    __syncthreads();
  }
  for (int64_t v = gtid(); v < n; v += gstride()) {
    if (lds) atomicAdd(&h[C[v]], 1);
    else atomicAdd(&s[C[v]], 1);
  }
  if (lds) {
    __syncthreads();
    for (int j = threadIdx.x; j < K0; j += kBlock)
      if (h[j]) atomicAdd(&s[j], h[j]);
  }
}

__global__ __launch_bounds__(kBlock) void k_sumsq(const int32_t* __restrict__ a, int64_t len,
                                                  int64_t* __restrict__ acc) {
  int64_t s = 0;
  for (int64_t j = gtid(); j < len; j += gstride()) {
    int64_t x = a[j];
    s += x * x;
  }
  s = block_sum<int64_t>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)acc, (unsigned long long)s);
}

// sum over labels l of partition i of |P_i l|^2, with |P_i l| = sum_x N_i(x, l)
__global__ __launch_bounds__(kBlock) void k_hist_sumsq(Tables t, int32_t K0,
                                                       int64_t* __restrict__ acc) {
  const int i = blockIdx.y;
  const int32_t Li = t.L[i];
  int64_t s = 0;
  for (int64_t l = gtid(); l < Li; l += gstride()) {
    int64_t h = 0;
    for (int32_t x = 0; x < K0; ++x) h += t.N[cell(t, i, x, (int32_t)l)];
    s += h * h;
  }
  s = block_sum<int64_t>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)acc, (unsigned long long)s);
}

// sum over vertices v and partitions i of N_i(C(v), l_i(v)): a cell whose
// count is c is met once by each of its c members, so this is the sum over
// cells of c^2, read from n k cells instead of the whole table
__global__ __launch_bounds__(kBlock) void k_gather_sumsq(const int32_t* __restrict__ C,
                                                         const int32_t* __restrict__ Lvm,
                                                         int64_t n, int32_t k, Tables t,
                                                         int64_t* __restrict__ acc) {
  int64_t s = 0;
  const uint32_t total = (uint32_t)(n * k);  // below 2^31
  for (uint32_t j = (uint32_t)gtid(); j < total; j += (uint32_t)gstride()) {
    const uint32_t v = j / (uint32_t)k;
    const int i = (int)(j - v * (uint32_t)k);
    s += count_of(t, i, C[v], Lvm[j]);
  }
  s = block_sum<int64_t>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)acc, (unsigned long long)s);
}

// ---- hashed tables ---------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_hash_clear(Tables t) {
  if (t.rows) {  // the keys (the caller zeroes the counts)
    for (int64_t j = gtid(); j <= (int64_t)t.hmask; j += gstride()) t.rkeys[j] = kHashEmpty;
    return;
  }
  uint4* H = reinterpret_cast<uint4*>(t.N);
  const uint4 empty = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
  for (int64_t j = gtid(); j <= (int64_t)t.hmask; j += gstride()) H[j] = empty;
}

// Cref[v] = label id of v in partition 0 (the reference of the row alignment)
__global__ __launch_bounds__(kBlock) void k_ref_labels(const int32_t* const* __restrict__ labels,
                                                       const int64_t* __restrict__ loff,
                                                       const int32_t* __restrict__ fmap, int64_t n,
                                                       int32_t* __restrict__ Cref) {
  const int32_t* p = labels[0];
  const int32_t* map = fmap + loff[0];
  for (int64_t v = gtid(); v < n; v += gstride()) Cref[v] = map[p[v]];
}

// rdist[v] = distinct label ids in v's row (the rows of a hashed-rows table
// v contributes to); *total += their sum.  k <= 64: a wave per vertex, lane
// i holding partition i, the first lane of each id counted by a ballot;
// else a thread per vertex.
__global__ __launch_bounds__(kBlock) void k_row_distinct(const int32_t* __restrict__ Lvm,
                                                         int64_t n, int32_t k,
                                                         uint8_t* __restrict__ rdist,
                                                         int64_t* __restrict__ total) {
  int64_t s = 0;
  if (k <= 64) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
    for (int64_t v = gtid() >> 6; v < n; v += nw) {
      const int32_t l = lane < k ? Lvm[v * k + lane] : -1;
      bool first = lane < k;
      for (int j = 0; j < k; ++j) {
        const int32_t o = __shfl(l, j, 64);
        if (j < lane && o == l) first = false;
      }
      const int32_t d = (int32_t)__popcll(__ballot(first));
      if (lane == 0) {
        rdist[v] = (uint8_t)min(d, 255);
        s += d;
      }
    }
  } else {
    for (int64_t v = gtid(); v < n; v += gstride()) {
      const int32_t* r = Lvm + v * k;
      int32_t d = 0;
      for (int i = 0; i < k; ++i) {
        const int32_t l = r[i];
        bool seen = false;
        for (int j = 0; j < i && !seen; ++j) seen = r[j] == l;
        d += !seen;
      }
      rdist[v] = (uint8_t)min(d, 255);
      s += d;
    }
  }
  s = block_sum<int64_t>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)total, (unsigned long long)s);
}

// Hashed rows from clusters of one vertex each (singletons): row (C[v], l)
// belongs to v alone, so its counts are stored, 1 at the partitions where
// v has label id l (the others stay at the zero they were filled with);
// each cell is written by one thread
__global__ __launch_bounds__(kBlock) void k_build_rows_single(const int32_t* __restrict__ C,
                                                              const int32_t* __restrict__ Lvm,
                                                              int64_t n, int32_t k, Tables t) {
  int32_t claimed = 0;
  const int64_t total = n * k;
  for (int64_t j = gtid(); j < total; j += gstride()) {
    const int64_t v = j / k;
    const int i = (int)(j - v * k);
    const uint32_t r = rslot(t, hkey(t, 0, C[v], Lvm[j]), claimed);
    t.N[(uint64_t)r * (uint64_t)k + (uint64_t)i] = 1;
  }
  flush_claims(t, claimed);
}

// Hashed rows: N[row(C[v], Lvm[v k + i]) k + i] += 1 for every (v, i),
// vertex-major (a vertex's partitions mostly share one row)
__global__ __launch_bounds__(kBlock) void k_build_rows(const int32_t* __restrict__ C,
                                                       const int32_t* __restrict__ Lvm, int64_t n,
                                                       int32_t k, Tables t) {
  flush_claims(t, rows_count(t, C, Lvm, n, k, gtid(), gstride()));
}

// hist[toff[i] + l] = |P_i l| (label ids in the hashed key space)
__global__ __launch_bounds__(kBlock) void k_label_hist(const int32_t* const* __restrict__ labels,
                                                       const int64_t* __restrict__ loff,
                                                       const int32_t* __restrict__ fmap,
                                                       const int64_t* __restrict__ toff, int64_t n,
                                                       int32_t* __restrict__ hist) {
  __shared__ int32_t h[kLdsHist];
  const int i = blockIdx.y;
  const int32_t* p = labels[i];
  const int32_t* map = fmap + loff[i];
  int32_t* hi = hist + toff[i];
  const int64_t Li = toff[i + 1] - toff[i];
  const bool lds = Li <= kLdsHist;  // few labels: count in LDS, flush once
  if (lds) {
    for (int64_t l = threadIdx.x; l < Li; l += kBlock) h[l] = 0;
    __syncthreads();
  }
  for (int64_t v = gtid(); v < n; v += gstride()) {
    const int32_t l = map[p[v]];
    if (lds) atomicAdd(&h[l], 1);
    else atomicAdd(&hi[l], 1);
  }
  if (lds) {
    __syncthreads();
    for (int64_t l = threadIdx.x; l < Li; l += kBlock)
      if (h[l]) atomicAdd(&hi[l], h[l]);
  }
}

// sum of squared slot counts
__global__ __launch_bounds__(kBlock) void k_slot_sumsq(Tables t, int64_t* __restrict__ acc) {
  const uint4* H = reinterpret_cast<const uint4*>(t.N);
  int64_t s = 0;
  for (int64_t j = gtid(); j <= (int64_t)t.hmask; j += gstride()) {
    const int64_t c = (int32_t)H[j].z;
    s += c * c;
  }
  s = block_sum<int64_t>(s);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)acc, (unsigned long long)s);
}

// ---- validation, output ----------------------------------------------------
// Every arc (v, u) must have a reverse arc (u, v): a search of u's row (work
// sum over u of deg(u)^2; a check, not on the solve path).
__global__ __launch_bounds__(kBlock) void k_check_symmetric(const int64_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            int64_t n, int32_t* __restrict__ err) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    bool ok = true;
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1] && ok; ++j) {
      const int32_t u = col[j];
      if (u == v) continue;
      bool found = false;
      for (int64_t p = row_ptr[u]; p < row_ptr[u + 1] && !found; ++p) found = col[p] == v;
      ok = found;
    }
    if (!ok) atomicOr(err, kErrGraph);
  }
}

__global__ __launch_bounds__(kBlock) void k_validate_csr(const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         int64_t n, int64_t nnz,
                                                         int32_t* __restrict__ err) {
  int bad = 0;
  if (gtid() == 0 && (row_ptr[0] != 0 || row_ptr[n] != nnz)) bad = 1;
  for (int64_t v = gtid(); v < n; v += gstride())
    if (row_ptr[v + 1] < row_ptr[v]) bad = 1;
  for (int64_t j = gtid(); j < nnz; j += gstride())
    if (col[j] < 0 || col[j] >= n) bad = 1;
  if (bad) atomicOr(err, kErrGraph);
}

__global__ __launch_bounds__(kBlock) void k_finish(const int32_t* __restrict__ C,
                                                   const int32_t* __restrict__ rawid, int64_t n,
                                                   int32_t* __restrict__ out) {
  for (int64_t v = gtid(); v < n; v += gstride()) out[v] = rawid[C[v]];
}

__global__ __launch_bounds__(kBlock) void k_count_nonzero(const int32_t* __restrict__ a, int64_t n,
                                                          int32_t* __restrict__ count) {
  int32_t c = 0;
  for (int64_t j = gtid(); j < n; j += gstride()) c += a[j] != 0;
  c = block_sum<int32_t>(c);
  if (threadIdx.x == 0 && c) atomicAdd(count, c);
}

__global__ __launch_bounds__(kBlock) void k_first_occurrence(const int32_t* __restrict__ in,
                                                             int64_t n, int32_t* __restrict__ first) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    int32_t x = in[v];
    if (__hip_atomic_load(&first[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > v)
      atomicMin(&first[x], (int32_t)v);
  }
}

__global__ __launch_bounds__(kBlock) void k_first_flags(const int32_t* __restrict__ in, int64_t n,
                                                        const int32_t* __restrict__ first,
                                                        int32_t* __restrict__ flags) {
  for (int64_t v = gtid(); v < n; v += gstride()) flags[v] = first[in[v]] == v;
}

__global__ __launch_bounds__(kBlock) void k_canonical_write(const int32_t* __restrict__ in,
                                                            int64_t n,
                                                            const int32_t* __restrict__ first,
                                                            const int32_t* __restrict__ rank,
                                                            int32_t* __restrict__ out) {
  for (int64_t v = gtid(); v < n; v += gstride()) out[v] = rank[first[in[v]]];
}

// ---- label alignment -----------------------------------------------------------
// Each label l of partition i has a home: the consensus cluster holding most
// of its vertices (ties to the smallest cluster).  Among the labels homed at
// cluster x, the largest (ties to the smallest label) takes id x; the others
// take ids K0, K0 + 1, ... in label order.  Any injective relabelling leaves
// every count unchanged; this one puts a vertex's labels and its cluster
// side by side in the interleaved table.
// The home of label l of partition i is its most frequent cluster in the
// sample, the smallest cluster id on ties.  Segment z of the clusters is
// searched by its own threads, which fold their (count, cluster) best into
// best[poff[i] + l] packed as count << 32 | ~cluster (zero-filled first).
__global__ __launch_bounds__(kBlock) void k_align_search(Tables b, int32_t K0, int32_t seg,
                                                         const int64_t* __restrict__ poff,
                                                         unsigned long long* __restrict__ best) {
  const int i = blockIdx.y;
  const int32_t Li = b.L[i];
  const int32_t x0 = (int32_t)blockIdx.z * seg, x1 = min(K0, x0 + seg);
  for (int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x; l < Li;
       l += (int64_t)gridDim.x * kBlock) {
    int32_t bx = x0, bc = -1;
    for (int32_t x = x0; x < x1; ++x) {
      const int32_t c = b.N[cell(b, i, x, (int32_t)l)];
      if (c > bc) {
        bc = c;
        bx = x;
      }
    }
    if (bc >= 0)
      atomicMax(&best[poff[i] + l],
                ((unsigned long long)(uint32_t)bc << 32) | (0xffffffffu - (uint32_t)bx));
  }
}

// home[p] and the label's claim key[p] (count << 32 | ~label) on its home,
// the largest claim per (partition, cluster) in win
__global__ __launch_bounds__(kBlock) void k_align_home(const int32_t* __restrict__ L,
                                                       int32_t K0,
                                                       const int64_t* __restrict__ poff,
                                                       uint64_t* __restrict__ win,
                                                       int32_t* __restrict__ home,
                                                       uint64_t* __restrict__ key) {
  const int i = blockIdx.y;
  for (int64_t l = gtid(); l < L[i]; l += gstride()) {
    const int64_t p = poff[i] + l;
    const uint64_t b = key[p];  // the packed best of k_align_search
    const int32_t bx = (int32_t)(0xffffffffu - (uint32_t)b);
    const uint32_t bc = (uint32_t)(b >> 32);
    const uint64_t kk = ((uint64_t)bc << 32) | (uint64_t)(0xffffffffu - (uint32_t)l);
    home[p] = bx;
    key[p] = kk;
    atomicMax((unsigned long long*)&win[(int64_t)i * K0 + bx], (unsigned long long)kk);
  }
}

__global__ __launch_bounds__(kBlock) void k_align_extra(const int32_t* __restrict__ L, int32_t K0,
                                                        const int64_t* __restrict__ poff,
                                                        const uint64_t* __restrict__ win,
                                                        const int32_t* __restrict__ home,
                                                        const uint64_t* __restrict__ key,
                                                        int32_t* __restrict__ extra) {
  const int i = blockIdx.y;
  for (int64_t l = gtid(); l < L[i]; l += gstride()) {
    const int64_t p = poff[i] + l;
    extra[p] = win[(int64_t)i * K0 + home[p]] != key[p];
  }
}

__global__ __launch_bounds__(kBlock) void k_align_assign(const int32_t* __restrict__ L,
                                                         int32_t K0,
                                                         const int64_t* __restrict__ poff,
                                                         const int32_t* __restrict__ home,
                                                         const int32_t* __restrict__ extra,
                                                         const int32_t* __restrict__ rank,
                                                         int32_t* __restrict__ amap,
                                                         int32_t* __restrict__ L2) {
  const int i = blockIdx.y;
  const int64_t b = poff[i];
  for (int64_t l = gtid(); l < L[i]; l += gstride()) {
    const int64_t p = b + l;
    amap[p] = extra[p] ? K0 + (rank[p] - rank[b]) : home[p];
  }
  if (gtid() == 0) L2[i] = K0 + (rank[poff[i + 1]] - rank[b]);
}

// ---- in-arc lists and arc clusters -------------------------------------------
__global__ __launch_bounds__(kBlock) void k_in_degree(const int32_t* __restrict__ col, int64_t nnz,
                                                      int32_t* __restrict__ indeg) {
  for (int64_t j = gtid(); j < nnz; j += gstride()) atomicAdd(&indeg[col[j]], 1);
}

__global__ __launch_bounds__(kBlock) void k_in_fill(const int32_t* __restrict__ col, int64_t nnz,
                                                    int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ in_pos) {
  for (int64_t j = gtid(); j < nnz; j += gstride())
    in_pos[atomicAdd(&cursor[col[j]], 1)] = (int32_t)j;
}

__global__ __launch_bounds__(kBlock) void k_arc_clusters(const int32_t* __restrict__ col,
                                                         int64_t nnz,
                                                         const int32_t* __restrict__ C,
                                                         int32_t* __restrict__ ac) {
  for (int64_t j = gtid(); j < nnz; j += gstride()) ac[j] = C[col[j]];
}

__global__ __launch_bounds__(kBlock) void k_copy_i32(const int32_t* __restrict__ src,
                                                     int32_t* __restrict__ dst, int64_t n) {
  for (int64_t j = gtid(); j < n; j += gstride()) dst[j] = src[j];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_narrow(const int32_t* __restrict__ src,
                                                   T* __restrict__ dst, int64_t n) {
  for (int64_t j = gtid(); j < n; j += gstride()) dst[j] = (T)src[j];
}

__global__ __launch_bounds__(kBlock) void k_dense_map(const int32_t* __restrict__ in, int64_t n,
                                                      const int32_t* __restrict__ scan,
                                                      int32_t* __restrict__ out) {
  const int32_t base = scan[0];
  for (int64_t v = gtid(); v < n; v += gstride()) out[v] = scan[in[v]] - base;
}

}  // namespace

// ---- launchers ---------------------------------------------------------------
int64_t scan_tmp_elems(int64_t len) { return (len + kScanTile - 1) / kScanTile + 2; }

void launch_scan(const int32_t* in, int32_t* out, int64_t len, int32_t* tmp, hipStream_t st) {
  // out[j] = sum_{t < j} in[t] for j in [0, len]; out may alias in
  int64_t nb = (len + kScanTile - 1) / kScanTile;
  if (nb < 1) nb = 1;
  k_scan_reduce<<<(unsigned)nb, kBlock, 0, st>>>(in, len, tmp);
  k_scan_top<<<1, kBlock, 0, st>>>(tmp, nb);
  k_scan_down<<<(unsigned)nb, kBlock, 0, st>>>(in, len, tmp, out);
}

void launch_label_max(const int32_t* const* dlabels, int32_t k, int64_t n, int32_t* maxlab,
                      int32_t* err, hipStream_t st) {
  // few workgroups: one atomic each per partition
  dim3 g(grid_for(n, kBlock * 16, 256), k);
  k_label_max<<<g, kBlock, 0, st>>>(dlabels, n, maxlab, err);
}

void launch_label_mark(const int32_t* const* dlabels, int32_t k, int64_t n, const int64_t* loff,
                       int32_t* flags, hipStream_t st) {
  dim3 g(grid_for(n, kBlock * 16, 2048), k);  // sixteen labels a thread
  k_label_mark<<<g, kBlock, 0, st>>>(dlabels, n, loff, flags);
}

void launch_label_counts(const int32_t* scan, const int64_t* loff, int32_t k, int32_t* Lc,
                         hipStream_t st) {
  k_label_counts<<<grid_for(k, kBlock), kBlock, 0, st>>>(scan, loff, k, Lc);
}

void launch_label_ids(const int32_t* scan, const int64_t* loff, int32_t k, int64_t max_span,
                      int32_t* fmap, hipStream_t st) {
  dim3 g(grid_for(max_span, kBlock, 256), k);
  k_label_ids<<<g, kBlock, 0, st>>>(scan, loff, fmap);
}

void launch_fmap_update(const int32_t* scan, const int64_t* loff, const int64_t* poff,
                        const int32_t* amap, int32_t k, int64_t max_span, int32_t* fmap,
                        hipStream_t st) {
  dim3 g(grid_for(max_span, kBlock, 256), k);
  k_fmap_update<<<g, kBlock, 0, st>>>(scan, loff, poff, amap, fmap);
}

void launch_align(const Tables& blocked, int32_t k, int32_t K0, int32_t maxL,
                  const int64_t* poff, int64_t total_labels, uint64_t* win, int32_t* home,
                  uint64_t* key, int32_t* extra, int32_t* rank, int32_t* scan_tmp,
                  int32_t* amap, int32_t* L2, hipStream_t st) {
  dim3 g(grid_for(maxL, kBlock, 256), k);
  k_fill_u64<<<grid_for((int64_t)k * K0, kBlock, 2048), kBlock, 0, st>>>(win, (int64_t)k * K0, 0ull);
  k_fill_u64<<<grid_for(total_labels, kBlock, 2048), kBlock, 0, st>>>(key, total_labels, 0ull);
  // enough segments of the clusters (at most 1024) to give the search
  // about 2^21 threads
  const int64_t lab_threads = (int64_t)((maxL + kBlock - 1) / kBlock) * kBlock * k;
  const int64_t nseg = std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(K0, 1024),
                           ((int64_t)1 << 21) / std::max<int64_t>(1, lab_threads)));
  const int32_t seg = (int32_t)((K0 + nseg - 1) / nseg);
  dim3 gs((unsigned)((maxL + kBlock - 1) / kBlock), (unsigned)k, (unsigned)((K0 + seg - 1) / seg));
  k_align_search<<<gs, kBlock, 0, st>>>(blocked, K0, seg, poff,
                                        reinterpret_cast<unsigned long long*>(key));
  k_align_home<<<g, kBlock, 0, st>>>(blocked.L, K0, poff, win, home, key);
  k_align_extra<<<g, kBlock, 0, st>>>(blocked.L, K0, poff, win, home, key, extra);
  launch_scan(extra, rank, total_labels, scan_tmp, st);
  k_align_assign<<<g, kBlock, 0, st>>>(blocked.L, K0, poff, home, extra, rank, amap, L2);
}

void launch_label_transpose(const int32_t* const* dlabels, int32_t k, int64_t n,
                            const int64_t* loff, const int32_t* fmap, int32_t* Lvm,
                            hipStream_t st) {
  int tv = 256;
  while (tv > 16 && (int64_t)(tv + 1) * k * 4 + 4 > 32 * 1024) tv >>= 1;
  if ((int64_t)(tv + 1) * k * 4 + 4 > 32 * 1024) {
    k_label_transpose_direct<<<grid_for(n * k, kBlock, 8192), kBlock, 0, st>>>(dlabels, k, n,
                                                                              loff, fmap, Lvm);
    return;
  }
  size_t lds = ((size_t)(tv + 1) * k + 1) * sizeof(int32_t);
  int64_t nb = (n + tv - 1) / tv;
  k_label_transpose<<<(unsigned)nb, kBlock, lds, st>>>(dlabels, k, n, loff, fmap, tv, Lvm);
}

void launch_cluster_mark(const int32_t* init, int64_t n, int32_t* flags, int32_t* err,
                         hipStream_t st) {
  k_cluster_mark<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(init, n, flags, err);
}

void launch_cluster_assign(const int32_t* init, int64_t n, const int32_t* cmap, int32_t* C,
                           int32_t* rawid, hipStream_t st) {
  k_cluster_assign<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(init, n, cmap, C, rawid);
}

void launch_iota(int32_t* a, int64_t n, hipStream_t st) {
  k_iota<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(a, n);
}

void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) k_fill_i32<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(a, n, v);
}

void launch_fill_u64(uint64_t* a, int64_t n, uint64_t v, hipStream_t st) {
  if (n > 0) k_fill_u64<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(a, n, v);
}

void launch_build(const int32_t* C, const int32_t* const* dlabels, const int64_t* loff,
                  const int32_t* fmap, int64_t n, int32_t k, int32_t K0, int32_t max_l, Tables t,
                  hipStream_t st, int64_t stride) {
  // enough workgroups per partition to fill the chip, few enough that the
  // LDS flush stays small next to the counting
  int64_t per_part = ((n + stride - 1) / stride + 4095) / 4096;  // about the sample size
  if (per_part > 64) per_part = 64;
  if (per_part < 1) per_part = 1;
  // LDS sized to the largest slice (up to 8 copies within 32 KiB; a slice
  // of up to kLdsHist entries alone), so that more workgroups share a CU
  const int64_t slice = (int64_t)K0 * max_l;
  int32_t cap = 0;
  if (!t.hashed && slice <= kLdsHist / 2)
    cap = (int32_t)(slice * std::min<int64_t>(8, (kLdsHist / 2) / std::max<int64_t>(slice, 1)));
  else if (!t.hashed && slice <= kLdsHist)
    cap = kLdsHist;
  dim3 g((unsigned)per_part, k);
  k_build<<<g, kBlock, (size_t)cap * sizeof(int32_t), st>>>(C, dlabels, loff, fmap, n, K0, t,
                                                           stride, cap);
}

void launch_sizes(const int32_t* C, int64_t n, int32_t K0, int32_t* s, hipStream_t st) {
  k_sizes<<<grid_for(n, kBlock * 16, 512), kBlock, 0, st>>>(C, n, K0, s);
}

void launch_objective0(const Tables& t, int32_t k, int32_t K0, int32_t maxL, const int32_t* s,
                       int64_t total_entries, const LabelHist& lh, const int32_t* C,
                       const int32_t* Lvm, int64_t n, int64_t* acc, hipStream_t st) {
  k_sumsq<<<grid_for(K0, kBlock, 1024), kBlock, 0, st>>>(s, K0, acc);
  if (total_entries <= n * (int64_t)k) {  // a small table: label sizes from its cells
    dim3 g(grid_for(maxL, kBlock, 64), k);
    k_hist_sumsq<<<g, kBlock, 0, st>>>(t, K0, acc + 1);
  } else {  // a large one: from the labels, n k reads
    launch_fill_i32(lh.hist, lh.total_labels, 0, st);
    dim3 g(grid_for(n, kBlock * 16, 64), k);
    k_label_hist<<<g, kBlock, 0, st>>>(lh.dlabels, lh.loff, lh.fmap, lh.lpoff, n, lh.hist);
    k_sumsq<<<grid_for(lh.total_labels, kBlock, 2048), kBlock, 0, st>>>(lh.hist, lh.total_labels,
                                                                        acc + 1);
  }
  if (Lvm && total_entries > 2 * n * (int64_t)k)
    k_gather_sumsq<<<grid_for(n * k, kBlock, 4096), kBlock, 0, st>>>(C, Lvm, n, k, t, acc + 2);
  else
    k_sumsq<<<grid_for(total_entries, kBlock, 2048), kBlock, 0, st>>>(t.N, total_entries, acc + 2);
}

void launch_hash_clear(Tables t, hipStream_t st) {
  k_hash_clear<<<grid_for((int64_t)t.hmask + 1, kBlock * 4, 4096), kBlock, 0, st>>>(t);
}

void launch_objective0_hashed(const Tables& t, const int32_t* const* dlabels, const int64_t* loff,
                              const int32_t* fmap, int64_t n, int32_t k, int32_t K0,
                              const int32_t* s, int64_t total_labels, int32_t* hist,
                              bool singletons, int64_t* acc, hipStream_t st) {
  k_sumsq<<<grid_for(K0, kBlock, 1024), kBlock, 0, st>>>(s, K0, acc);
  launch_fill_i32(hist, total_labels, 0, st);
  dim3 g(grid_for(n, kBlock * 16, 64), k);
  k_label_hist<<<g, kBlock, 0, st>>>(dlabels, loff, fmap, t.toff, n, hist);
  k_sumsq<<<grid_for(total_labels, kBlock, 2048), kBlock, 0, st>>>(hist, total_labels, acc + 1);
  const int64_t slots = (int64_t)t.hmask + 1;
  if (singletons)
    launch_fill_u64(reinterpret_cast<uint64_t*>(acc + 2), 1, (uint64_t)(n * (int64_t)k), st);
  else if (t.rows)
    k_sumsq<<<grid_for(slots * k, kBlock, 4096), kBlock, 0, st>>>(t.N, slots * k, acc + 2);
  else
    k_slot_sumsq<<<grid_for(slots, kBlock * 4, 4096), kBlock, 0, st>>>(t, acc + 2);
}

void launch_check_symmetric(const int64_t* row_ptr, const int32_t* col, int64_t n,
                            int32_t* err, hipStream_t st) {
  if (n > 0) k_check_symmetric<<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(row_ptr, col, n, err);
}

void launch_in_degree(const int32_t* col, int64_t nnz, int32_t* indeg, hipStream_t st) {
  if (nnz > 0) k_in_degree<<<grid_for(nnz, kBlock, 4096), kBlock, 0, st>>>(col, nnz, indeg);
}

void launch_in_fill(const int32_t* col, int64_t nnz, int32_t* cursor, int32_t* in_pos,
                    hipStream_t st) {
  if (nnz > 0) k_in_fill<<<grid_for(nnz, kBlock, 4096), kBlock, 0, st>>>(col, nnz, cursor, in_pos);
}

void launch_arc_clusters(const int32_t* col, int64_t nnz, const int32_t* C, int32_t* ac,
                         hipStream_t st) {
  if (nnz > 0) k_arc_clusters<<<grid_for(nnz, kBlock, 4096), kBlock, 0, st>>>(col, nnz, C, ac);
}

void launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t st) {
  if (n > 0) k_copy_i32<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(src, dst, n);
}

void launch_narrow(const int32_t* src, void* dst, int32_t bytes, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int g = grid_for(n, kBlock, 2048);
  if (bytes == 1) k_narrow<uint8_t><<<g, kBlock, 0, st>>>(src, (uint8_t*)dst, n);
  else if (bytes == 2) k_narrow<uint16_t><<<g, kBlock, 0, st>>>(src, (uint16_t*)dst, n);
  else k_narrow<int32_t><<<g, kBlock, 0, st>>>(src, (int32_t*)dst, n);
}

void launch_validate_csr(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* err, hipStream_t st) {
  k_validate_csr<<<grid_for(nnz > n ? nnz : n, kBlock, 2048), kBlock, 0, st>>>(row_ptr, col, n,
                                                                               nnz, err);
}

void launch_finish(const int32_t* C, const int32_t* rawid, int64_t n, int32_t* out,
                   hipStream_t st) {
  k_finish<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(C, rawid, n, out);
}

void launch_count_nonzero(const int32_t* a, int64_t n, int32_t* count, hipStream_t st) {
  k_count_nonzero<<<grid_for(n, kBlock, 1024), kBlock, 0, st>>>(a, n, count);
}

void launch_first_occurrence(const int32_t* in, int64_t n, int32_t* first, hipStream_t st) {
  k_first_occurrence<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(in, n, first);
}

void launch_first_flags(const int32_t* in, int64_t n, const int32_t* first, int32_t* flags,
                        hipStream_t st) {
  k_first_flags<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(in, n, first, flags);
}

void launch_canonical_write(const int32_t* in, int64_t n, const int32_t* first,
                            const int32_t* rank, int32_t* out, hipStream_t st) {
  k_canonical_write<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(in, n, first, rank, out);
}

void launch_dense_map(const int32_t* in, int64_t n, const int32_t* scan, int32_t* out,
                      hipStream_t st) {
  k_dense_map<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(in, n, scan, out);
}

void launch_ref_labels(const int32_t* const* dlabels, const int64_t* loff, const int32_t* fmap,
                       int64_t n, int32_t* Cref, hipStream_t st) {
  if (n > 0) k_ref_labels<<<grid_for(n, kBlock, 2048), kBlock, 0, st>>>(dlabels, loff, fmap, n, Cref);
}

void launch_row_distinct(const int32_t* Lvm, int64_t n, int32_t k, uint8_t* rdist, int64_t* total,
                         hipStream_t st) {
  if (n > 0) k_row_distinct<<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(Lvm, n, k, rdist, total);
}

void launch_build_rows_single(const int32_t* C, const int32_t* Lvm, int64_t n, int32_t k,
                              Tables t, hipStream_t st) {
  if (n > 0)
    k_build_rows_single<<<grid_for(n * k, kBlock, 8192), kBlock, 0, st>>>(C, Lvm, n, k, t);
}

void launch_build_rows(const int32_t* C, const int32_t* Lvm, int64_t n, int32_t k, Tables t,
                       hipStream_t st) {
  if (n > 0) k_build_rows<<<grid_for(n * k, kBlock, 8192), kBlock, 0, st>>>(C, Lvm, n, k, t);
}

}  // namespace mcc
