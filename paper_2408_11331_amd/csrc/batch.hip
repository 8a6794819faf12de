// Batched consensus: many independent instances in one persistent launch.
//
// Each workgroup pops an instance from a queue (largest estimated work
// first) and runs the whole method on it: consensus-cluster compaction,
// vertex-major label rows, contingency tables, and the synchronous pass
// loop of the single-instance path (score every vertex against the frozen
// partition, apply the batch, keep it if the objective drops, else the
// conflict-free owner subset), with workgroup barriers in place of kernel
// boundaries.  Per-instance state lives in a workspace slot owned by the
// workgroup for the duration of the instance.  An instance that exceeds a
// slot's capacities is reported back and solved by the single-instance
// path, so every output equals the single-instance output bit for bit.
//
// The workgroup keeps many memory accesses in flight: sweeps take several
// elements per thread before waiting, label values small enough serve
// directly as table columns (any injective relabelling leaves every count
// unchanged, so no compaction pass), each partition's table slice and label
// sizes are histogrammed in LDS in one pass over its labels, scoring walks
// tiles of 256 vertices (arcs spread over all threads, candidate sets in
// LDS, probes by 16-lane groups with four pairs in flight), and the apply
// spreads each proposal's partitions over 16 lanes.
#include "batch.h"

namespace mcc {

namespace {

constexpr int kBatchLds = 8192;  // int32 entries of a table slice (or sizes) in LDS
constexpr int kLabLds = 1024;    // label values whose sizes are counted in LDS
constexpr int kSweep = 8;        // elements per thread in flight in the sweeps
constexpr int32_t kNone = -1;
constexpr int32_t kDefer = -3;   // the tile scorer left the vertex to the group scorer
constexpr int64_t kGainBias = (int64_t)1 << 33;

// tile scorer geometry (as in the single-instance tiled scorer)
constexpr int kArcChunk = 1024;
constexpr int kSetSlots = 2048;
constexpr int kSetProbe = 64;
constexpr int kPairMax = kSetSlots + kBlock;
constexpr int kProbeLanes = 16;
constexpr int kProbeRegs = 64 / kProbeLanes;
constexpr int kProbeBatch = 4;

__device__ inline uint64_t owner_key(int64_t gain, int64_t v) {
  return ((uint64_t)(gain + kGainBias) << 31) | (uint64_t)v;
}

template <int G>
__device__ inline int32_t group_min(int32_t x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, G));
  return x;
}

template <int G>
__device__ inline int32_t group_sum(int32_t x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

// Contingency counts of an instance: int32, or int16 when the instance has
// fewer than 2^15 vertices (every count is at most n), which halves the
// table that every probe reads.  Two int16 counts share a 32-bit word;
// an atomic addition to one of them adds to the word, shifted to its half:
// a count never passes 2^15 - 1 or drops below 0, so no carry or borrow
// reaches the other half.
template <typename T>
struct Counts {
  T* p;
  __device__ int32_t get(int64_t j) const { return p[j]; }
  __device__ void set(int64_t j, int32_t v) const { p[j] = (T)v; }
  __device__ int32_t add(int64_t j, int32_t d) const {
    if constexpr (sizeof(T) == 4) {
      return atomicAdd(reinterpret_cast<int32_t*>(p) + j, d);
    } else {
      const uintptr_t a = reinterpret_cast<uintptr_t>(p + j);
      int32_t* word = reinterpret_cast<int32_t*>(a & ~(uintptr_t)3);
      const int sh = (a & 2) ? 16 : 0;
      const int32_t old = atomicAdd(word, (int32_t)((uint32_t)d << sh));
      return (int32_t)(int16_t)((uint32_t)old >> sh);
    }
  }
};

// workgroup reductions (all threads call; result valid in every thread)
template <typename T, typename Op>
__device__ T wg_reduce(T x, Op op, T* scratch /* kBlock / 64 */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = op(x, __shfl_xor(x, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = x;
  __syncthreads();
  T r = scratch[0];
#pragma unroll
  for (int j = 1; j < kBlock / 64; ++j) r = op(r, scratch[j]);
  __syncthreads();
  return r;
}

struct Max32 {
  __device__ int32_t operator()(int32_t a, int32_t b) const { return a > b ? a : b; }
};
struct Min32 {
  __device__ int32_t operator()(int32_t a, int32_t b) const { return a < b ? a : b; }
};
struct Add64 {
  __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
};

// In-place exclusive scan of a[0..len) by one workgroup (kSweep consecutive
// elements per thread per chunk); returns the total.
__device__ int32_t wg_scan(int32_t* a, int64_t len) {
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < len; b0 += (int64_t)kBlock * kSweep) {
    const int64_t base = b0 + (int64_t)threadIdx.x * kSweep;
    int32_t x[kSweep], loc = 0;
#pragma unroll
    for (int u = 0; u < kSweep; ++u) {
      x[u] = base + u < len ? a[base + u] : 0;
      loc += x[u];
    }
    int32_t tot;
    int32_t run = carry + block_exclusive_scan(loc, &tot);
#pragma unroll
    for (int u = 0; u < kSweep; ++u) {
      if (base + u < len) a[base + u] = run;
      run += x[u];
    }
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// One scoring pass over the instance (or only over the vertices the tile
// scorer deferred): G lanes per vertex, kBlock / G vertices at a time.
// Candidates are taken in increasing cluster id by repeated group minima, so the result does not depend on G.  Kept out of
// line: inlined, the five variants share one register allocation and the
// kernel loses a wave per SIMD.
template <int G, typename T>
__device__ __attribute__((noinline)) void score_pass(int64_t n_, int32_t k_, const int64_t* row_ptr,
                           const int32_t* col, bool literal, const int32_t* C,
                           const int32_t* Lvm, const T* N, const int32_t* s,
                           int32_t Lmax, int32_t* prop,
                           int64_t* dprop, bool deferred_only, int64_t* evals_out,
                           int32_t* np_out) {
  constexpr int R = 8;  // arc registers per lane before re-reading memory
  constexpr int32_t kInf = 0x7fffffff;
  constexpr int NG = kBlock / G;
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  const int64_t n = n_;
  const int32_t k = k_;
  int64_t evals = 0;
  int32_t np = 0;
  for (int64_t v = grp; v < n; v += NG) {
    if (deferred_only && prop[v] != kDefer) continue;
    const int32_t cv = C[v];
    const int64_t beg = row_ptr[v], end = row_ptr[v + 1];
    const bool fits = end - beg <= (int64_t)G * R;
    int32_t xr[R];
    if (fits) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t j = beg + r * G + lane;
        xr[r] = kInf;
        if (j < end) {
          const int32_t cu = C[col[j]];
          if (cu != cv) xr[r] = cu;
        }
      }
    }
    const int32_t* row = Lvm + v * k;
    auto agree = [&](int32_t y) -> int32_t {
      int32_t sum = 0;
      const int64_t base = (int64_t)y * Lmax;
      for (int i = lane; i < k; i += G) sum += N[(base + row[i]) * k + i];
      return group_sum<G>(sum);
    };
    int32_t last = -1, ncand = 0, bestx = kNone;
    int64_t bestd = 0, s_own = -1;
    const int64_t sc = s[cv];
    for (;;) {
      int32_t mn = kInf;
      if (fits) {
#pragma unroll
        for (int r = 0; r < R; ++r) mn = min(mn, xr[r]);
      } else {
        for (int64_t j = beg + lane; j < end; j += G) {
          const int32_t cu = C[col[j]];
          if (cu != cv && cu > last && cu < mn) mn = cu;
        }
      }
      mn = group_min<G>(mn);
      if (mn == kInf) break;
      if (s_own < 0) s_own = agree(cv);
      const int64_t sx = agree(mn);
      int64_t d = 2 * (s_own - sx) + (int64_t)k * ((int64_t)s[mn] - sc - 1);
      if (literal) d += k;
      if (ncand == 0 || d < bestd) {
        bestd = d;
        bestx = mn;
      }
      ++ncand;
      last = mn;
      if (fits) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (xr[r] == mn) xr[r] = kInf;
      }
    }
    if (lane == 0) {
      evals += ncand;
      const bool pp = ncand > 0 && bestd < 0;
      prop[v] = pp ? bestx : kNone;
      if (pp) {
        dprop[v] = bestd;
        ++np;
      }
    }
  }
  *evals_out = evals;
  *np_out = np;
}


// LDS of one workgroup: the set-up histograms and the tile scorer's state
// are never live at the same time.
struct SetupLds {
  int32_t h[kBatchLds];   // sizes, then one partition's table slice
  int32_t lab[kLabLds];   // one partition's label sizes
};
struct TileLds {
  int32_t off[kBlock + 1];
  int32_t c[kBlock];
  int32_t nc[kBlock];
  int32_t def[kBlock];
  int32_t cur[kBlock];
  int32_t set[kSetSlots];
  int32_t cl[kPairMax];   // pair keys (vertex << 24 | cluster), a run per vertex
  int32_t S[kPairMax];    // agreement sum of each pair
  int32_t np;
};
union BatchLds {
  SetupLds su;
  TileLds ti;
};

// One scoring pass by tiles of kBlock vertices (k <= 64 or not): candidate
// sets in LDS, probes by 16-lane groups.  Vertices whose candidates do not
// fit the set or the pair arrays are marked kDefer for the group scorer.
template <typename T>
__device__ __attribute__((noinline)) void tile_pass(int64_t n_, int32_t k_, const int64_t* row_ptr,
                                                   const int32_t* col, bool literal,
                                                   const int32_t* C, const int32_t* Lvm,
                          const T* N, const int32_t* s, int32_t Ls, int32_t* prop,
                          int64_t* dprop, TileLds& L, int64_t* evals_out, int32_t* np_out,
                          int32_t* ndef_out) {
  const int t = threadIdx.x;
  const int64_t n = n_;
  const int32_t k = k_;
  const bool kfits = k <= kProbeRegs * kProbeLanes;
  const int g = t / kProbeLanes, lane = t % kProbeLanes;
  int64_t evals = 0;
  int32_t np = 0, ndef = 0;
  const int64_t ntiles = (n + kBlock - 1) / kBlock;
  for (int64_t tile = 0; tile < ntiles; ++tile) {
    const int64_t v0 = tile * kBlock;
    const int nv = (int)min((int64_t)kBlock, n - v0);
    const int64_t a0 = row_ptr[v0];
    for (int j = t; j <= nv; j += kBlock) L.off[j] = (int32_t)(row_ptr[v0 + j] - a0);
    L.c[t] = t < nv ? C[v0 + t] : -1;
    L.nc[t] = 0;
    L.def[t] = 0;
    for (int j = t; j < kSetSlots; j += kBlock) L.set[j] = -1;
    __syncthreads();
    const int32_t A = L.off[nv];
    constexpr int U = kArcChunk / kBlock;
    int32_t hn[U];  // the next chunk's heads, loaded while this one is processed
#pragma unroll
    for (int r = 0; r < U; ++r) hn[r] = t * U + r < A ? col[a0 + t * U + r] : 0;
    for (int32_t cb = 0; cb < A; cb += kArcChunk) {
      const int32_t jt = cb + t * U;  // tile-relative index of the thread's first arc
      int32_t hd[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        hd[r] = hn[r];
        const int32_t jn = jt + kArcChunk + r;
        hn[r] = jn < A ? col[a0 + jn] : 0;
      }
      int lo = 0;
      if (jt < A) {
        int hi = nv - 1;  // tail: the last vertex whose row starts at or before jt
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (L.off[mid] <= jt) lo = mid;
          else hi = mid - 1;
        }
      }
      int tl[U];
      int32_t cu[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        tl[r] = -1;
        if (jt + r >= A) continue;
        while (L.off[lo + 1] <= jt + r) ++lo;
        tl[r] = lo;
      }
#pragma unroll
      for (int r = 0; r < U; ++r) cu[r] = tl[r] >= 0 ? C[hd[r]] : -1;
      int32_t prev = -1;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (tl[r] < 0) continue;
        const int tv = tl[r];
        const int32_t x = cu[r];
        if (x == L.c[tv]) continue;  // own cluster (and self-loops)
        const int32_t key = (tv << 24) | x;
        if (key == prev) continue;
        prev = key;
        uint32_t h = ((uint32_t)key * 2654435761u) >> 21;  // 11 bits: kSetSlots
        bool placed = false;
        for (int q = 0; q < kSetProbe; ++q) {
          int32_t cur = L.set[h];
          if (cur == -1) cur = atomicCAS(&L.set[h], -1, key);
          if (cur == -1) {
            atomicAdd(&L.nc[tv], 1);
            placed = true;
            break;
          }
          if (cur == key) {
            placed = true;
            break;
          }
          h = (h + 1) & (kSetSlots - 1);
        }
        if (!placed) L.def[tv] = 1;
      }
    }
    __syncthreads();
    const int nc = L.nc[t];
    bool def = t < nv && L.def[t];
    bool is_b = t < nv && nc > 0 && !def;
    int32_t npairs;
    const int32_t coff = block_exclusive_scan(is_b ? nc + 1 : 0, &npairs);
    if (t == 0) L.np = npairs;
    __syncthreads();
    if (is_b && coff + nc + 1 > kPairMax) {  // a run past the pair arrays
      is_b = false;
      def = true;
      L.def[t] = 1;
      atomicMin(&L.np, coff);
    }
    if (t < nv) {
      const int64_t v = v0 + t;
      if (def) {
        prop[v] = kDefer;
        ++ndef;
      } else if (nc == 0) {
        prop[v] = kNone;
      } else {
        evals += nc;
      }
    }
    L.cur[t] = coff + 1;
    if (is_b) L.cl[coff] = (t << 24) | L.c[t];
    __syncthreads();
    npairs = L.np;
    for (int h = t; h < kSetSlots; h += kBlock) {
      const int32_t key = L.set[h];
      if (key == -1) continue;
      const int tv = (int)((uint32_t)key >> 24);
      if (L.def[tv]) continue;
      L.cl[atomicAdd(&L.cur[tv], 1)] = key;
    }
    __syncthreads();
    // probes: 16-lane groups, kProbeBatch pairs each, lanes over the
    // partitions; the next round's label rows are loaded before this
    // round's probes
    constexpr int kStride = (kBlock / kProbeLanes) * kProbeBatch;
    if (kfits) {
      int32_t xs[kProbeBatch], lab[kProbeBatch][kProbeRegs];
      auto fetch = [&](int p, int32_t* xq, int32_t (*lq)[kProbeRegs]) {
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          xq[q] = -1;
          int64_t row = 0;
          if (p + q < npairs) {
            const int32_t key = L.cl[p + q];
            xq[q] = key & 0xffffff;
            row = (v0 + (int)((uint32_t)key >> 24)) * (int64_t)k;
          }
#pragma unroll
          for (int r = 0; r < kProbeRegs; ++r) {
            const int i = lane + r * kProbeLanes;
            lq[q][r] = (xq[q] >= 0 && i < k) ? Lvm[row + i] : 0;
          }
        }
      };
      int p0 = g * kProbeBatch;
      fetch(p0, xs, lab);
      for (; p0 < npairs; p0 += kStride) {
        int32_t xn[kProbeBatch], labn[kProbeBatch][kProbeRegs];
        fetch(p0 + kStride, xn, labn);
        int32_t sums[kProbeBatch];
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          int32_t sum = 0;
#pragma unroll
          for (int r = 0; r < kProbeRegs; ++r) {
            const int i = lane + r * kProbeLanes;
            if (xs[q] >= 0 && i < k) sum += N[((int64_t)xs[q] * Ls + lab[q][r]) * k + i];
          }
          sums[q] = sum;
        }
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          const int32_t sq = group_sum<kProbeLanes>(sums[q]);
          if (lane == 0 && xs[q] >= 0) L.S[p0 + q] = sq;
          xs[q] = xn[q];
#pragma unroll
          for (int r = 0; r < kProbeRegs; ++r) lab[q][r] = labn[q][r];
        }
      }
    } else {
      for (int p0 = g * kProbeBatch; p0 < npairs; p0 += kStride) {
        int32_t sums[kProbeBatch], xs[kProbeBatch];
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          int32_t sum = 0;
          xs[q] = -1;
          if (p0 + q < npairs) {
            const int32_t key = L.cl[p0 + q];
            xs[q] = key & 0xffffff;
            const int64_t row = (v0 + (int)((uint32_t)key >> 24)) * (int64_t)k;
            for (int i = lane; i < k; i += kProbeLanes)
              sum += N[((int64_t)xs[q] * Ls + Lvm[row + i]) * k + i];
          }
          sums[q] = sum;
        }
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          const int32_t sq = group_sum<kProbeLanes>(sums[q]);
          if (lane == 0 && xs[q] >= 0) L.S[p0 + q] = sq;
        }
      }
    }
    __syncthreads();
    if (is_b) {
      const int64_t v = v0 + t;
      const int32_t c = L.c[t];
      const int64_t s_own = L.S[coff];
      const int64_t scz = s[c];
      int64_t bestd = 0;
      int32_t bestx = kNone;
      for (int j = coff + 1; j <= coff + nc; ++j) {
        const int32_t x = L.cl[j] & 0xffffff;
        int64_t d = 2 * (s_own - (int64_t)L.S[j]) + (int64_t)k * ((int64_t)s[x] - scz - 1);
        if (literal) d += k;
        if (bestx == kNone || d < bestd || (d == bestd && x < bestx)) {
          bestd = d;
          bestx = x;
        }
      }
      const bool pp = bestd < 0;
      prop[v] = pp ? bestx : kNone;
      if (pp) {
        dprop[v] = bestd;
        ++np;
      }
    }
    __syncthreads();
  }
  *evals_out = evals;
  *np_out = np;
  *ndef_out = ndef;
}

// The moves of one set of proposals, sign d (+1 apply, -1 undo), with the
// partitions of each proposal spread over a 16-lane group.  sel(v, to)
// selects the proposals.  Returns this thread's share of the change of the
// sums of squares (N part in *dn2, sizes in *ds2) and of the moves.
// The moves of one set of proposals, sign d (+1 apply, -1 undo), with the
// partitions of each proposal spread over a 16-lane group.  mode selects
// the proposals: 0 all, 1 those owning both their clusters (owner keys).
// Adds this thread's share of the change of the sums of squares (N part in
// *dn2, sizes in *ds2) and returns its count of moves.
template <typename T>
__device__ __attribute__((noinline)) int32_t apply_moves(
    int64_t n, int32_t k, const int32_t* prop, const int32_t* C, const int32_t* Lvm, Counts<T> N,
    int32_t* s, int32_t Ls, int32_t d, int mode, const uint64_t* owner, const int64_t* dprop,
    int64_t* dn2, int64_t* ds2) {
  constexpr int kL = 16;
  const int lane = threadIdx.x & 63, grp = lane / kL, gl = lane % kL;
  const int wave = threadIdx.x >> 6;
  int32_t moved = 0;
  int64_t n2 = 0, s2 = 0;
  for (int64_t v0 = (int64_t)wave * 64; v0 < n; v0 += kBlock) {
    const int64_t v = v0 + lane;
    const int32_t p = v < n ? prop[v] : kNone;
    bool take = v < n && p >= 0;
    if (take && mode == 1) {
      const uint64_t key = owner_key(dprop[v], v);
      take = owner[C[v]] == key && owner[p] == key;
    }
    uint64_t mask = __ballot(take);
    while (mask) {
      uint64_t m = mask;  // this group's proposal: the grp-th selected vertex
      for (int q = 0; q < grp; ++q) m &= m - 1;
      const int b = m ? __ffsll((unsigned long long)m) - 1 : -1;
      for (int q = 0; q < 64 / kL; ++q) mask &= mask - 1;
      const int32_t to = __shfl(p, b < 0 ? 0 : b, 64);
      if (b < 0) continue;
      const int64_t w = v0 + b;
      const int32_t from = C[w];
      const int32_t* row = Lvm + w * k;
      for (int i = gl; i < k; i += kL) {
        const int32_t l = row[i];
        const int32_t o1 = N.add(((int64_t)to * Ls + l) * k + i, d);
        const int32_t o2 = N.add(((int64_t)from * Ls + l) * k + i, -d);
        n2 += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
      }
      if (gl == 0) {
        const int32_t o1 = atomicAdd(&s[to], d);
        const int32_t o2 = atomicAdd(&s[from], -d);
        s2 += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
        ++moved;
      }
    }
  }
  *dn2 += n2;
  *ds2 += s2;
  return moved;
}

// Shared state of one instance between the phases (written by thread 0 or
// identically by all threads, read after a barrier).
struct InstState {
  int64_t acc;     // objective terms summed so far
  int32_t K0;      // consensus clusters
  int32_t Ls;      // label ids lie in [0, Ls)
  int32_t status;  // 0, kBatchTooBig or kBatchInvalid
  int32_t pad;
};

// Consensus clusters: dense ids in order of the initial ids, sizes, owners.
__device__ __attribute__((noinline)) void phase_clusters(
    int64_t n, int32_t k, const int32_t* init, int32_t* flags, int32_t* C, int32_t* rawid,
    int32_t* s, uint64_t* owner, int32_t* h, int32_t* r32, int64_t* r64, InstState* st) {
  const int t = threadIdx.x;
  int32_t K0;
  if (init) {
    for (int64_t x = t; x <= n; x += kBlock) flags[x] = 0;
    __syncthreads();
    int32_t bad = 0;
    for (int64_t v0 = t; v0 < n; v0 += (int64_t)kBlock * kSweep) {
      int32_t xs[kSweep];
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        xs[u] = v < n ? init[v] : 0;
      }
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        if (v0 + (int64_t)u * kBlock >= n) continue;
        if (xs[u] < 0 || xs[u] >= n) bad = 1;
        else flags[xs[u]] = 1;
      }
    }
    bad = wg_reduce(bad, Max32(), r32);
    if (bad) {
      if (t == 0) st->status = kBatchInvalid;
      __syncthreads();
      return;
    }
    K0 = wg_scan(flags, n);
    if (t == 0) flags[n] = K0;
    __syncthreads();
    for (int64_t v0 = t; v0 < n; v0 += (int64_t)kBlock * kSweep) {
      int32_t xs[kSweep];
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        xs[u] = v < n ? init[v] : 0;
      }
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        if (v >= n) continue;
        C[v] = flags[xs[u]];
        if (flags[v + 1] > flags[v]) rawid[flags[v]] = (int32_t)v;
      }
    }
  } else {
    K0 = (int32_t)n;
    for (int64_t v = t; v < n; v += kBlock) {
      C[v] = (int32_t)v;
      rawid[v] = (int32_t)v;
    }
  }
  __syncthreads();
  const bool lds_sizes = K0 <= kBatchLds;
  for (int64_t x = t; x < K0; x += kBlock) {
    owner[x] = ~0ull;
    if (lds_sizes) h[x] = 0;
    else s[x] = 0;
  }
  __syncthreads();
  for (int64_t v = t; v < n; v += kBlock) {
    if (lds_sizes) atomicAdd(&h[C[v]], 1);
    else atomicAdd(&s[C[v]], 1);
  }
  __syncthreads();
  int64_t acc = 0;
  for (int64_t x = t; x < K0; x += kBlock) {
    const int32_t sx = lds_sizes ? h[x] : s[x];
    if (lds_sizes) s[x] = sx;
    acc += (int64_t)k * sx * sx;
  }
  acc = wg_reduce(acc, Add64(), r64);
  if (t == 0) {
    st->K0 = K0;
    st->acc = acc;
  }
  __syncthreads();
}

// Vertex-major label rows and the label range, in one sweep.
__device__ __attribute__((noinline)) void phase_rows(int64_t n, int32_t k,
                                                    const int32_t* const* labels, int32_t* Lvm,
                                                    int32_t* r32, InstState* st) {
  const int t = threadIdx.x;
  int32_t lmax = -1, lmin = 0;
  for (int64_t v = t; v < n; v += kBlock) {
    int32_t* row = Lvm + v * k;
    for (int i0 = 0; i0 < k; i0 += kSweep) {
      int32_t x[kSweep];
#pragma unroll
      for (int u = 0; u < kSweep; ++u) x[u] = i0 + u < k ? labels[i0 + u][v] : 0;
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        if (i0 + u >= k) continue;
        row[i0 + u] = x[u];
        lmax = max(lmax, x[u]);
        lmin = min(lmin, x[u]);
      }
    }
  }
  lmax = wg_reduce(lmax, Max32(), r32);
  lmin = wg_reduce(lmin, Min32(), r32);
  if (t == 0) {
    st->Ls = lmax + 1;  // label values are the table's label ids
    if (lmin < 0) st->status = kBatchInvalid;
  }
  __syncthreads();
}

// Contingency table N[(x * Ls + l) * k + i], one partition at a time: its
// K0 x Ls slice and its label sizes histogrammed in LDS in one pass over its
// labels (global counters when they do not fit), written once; the
// objective's sums of squares from the same counts.
template <typename T>
__device__ __attribute__((noinline)) void phase_tables(
    int64_t n, int32_t k, const int32_t* const* labels, const int32_t* C, Counts<T> N,
    int32_t* flags, int32_t* h, int32_t* lab, int64_t* r64, InstState* st) {
  const int t = threadIdx.x;
  const int32_t K0 = st->K0, Ls = st->Ls;
  const int64_t slice = (int64_t)K0 * Ls;
  const bool lds_tab = slice <= kBatchLds;
  const bool lds_lab = Ls <= kLabLds;
  int32_t* labh = lds_lab ? lab : flags;
  int64_t acc = 0;
  for (int i = 0; i < k; ++i) {
    const int32_t* p = labels[i];
    for (int64_t j = t; j < slice; j += kBlock) {
      if (lds_tab) h[j] = 0;
      else N.set(j * k + i, 0);
    }
    for (int32_t l = t; l < Ls; l += kBlock) labh[l] = 0;
    __syncthreads();
    for (int64_t v0 = t; v0 < n; v0 += (int64_t)kBlock * kSweep) {
      int32_t ls[kSweep], cs[kSweep];
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        ls[u] = v < n ? p[v] : 0;
        cs[u] = v < n ? C[v] : 0;
      }
#pragma unroll
      for (int u = 0; u < kSweep; ++u) {
        if (v0 + (int64_t)u * kBlock >= n) continue;
        const int64_t j = (int64_t)cs[u] * Ls + ls[u];
        if (lds_tab) atomicAdd(&h[j], 1);
        else N.add(j * k + i, 1);
        atomicAdd(&labh[ls[u]], 1);
      }
    }
    __syncthreads();
    for (int64_t j = t; j < slice; j += kBlock) {
      const int32_t c = lds_tab ? h[j] : N.get(j * k + i);
      if (lds_tab) N.set(j * k + i, c);
      acc -= 2 * (int64_t)c * c;
    }
    for (int32_t l = t; l < Ls; l += kBlock) acc += (int64_t)labh[l] * labh[l];
    __syncthreads();
  }
  acc = wg_reduce(acc, Add64(), r64);
  if (t == 0) st->acc += acc;
  __syncthreads();
}

// Tables, the pass loop and the output of one instance whose set-up
// (clusters, label rows, label range) is done; T is the count type.
template <typename T>
__device__ __attribute__((noinline)) void run_instance(
    const BatchArgs& b, const BatchInst& in, int64_t n, int32_t k, Counts<T> N, int32_t* C,
    int32_t* rawid, int32_t* prop, int64_t* dprop, int32_t* s, uint64_t* owner, int32_t* Lvm,
    int32_t* flags, BatchLds& L, int32_t* s_r32, int64_t* s_r64, InstState* S, BatchRes& res) {
  const int t = threadIdx.x;
  phase_tables<T>(n, k, in.labels, C, N, flags, L.su.h, L.su.lab, s_r64, S);
  const int32_t K0 = S->K0, Ls = S->Ls;
  int64_t O = S->acc;
  res.objective_init = O;

  // ---- pass loop ----
  for (;;) {
    int64_t evals = 0, evals2 = 0;
    int32_t np = 0, np2 = 0, ndef = 0;
    const bool lit = b.literal != 0;
    tile_pass<T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, L.ti, &evals, &np,
              &ndef);
    ndef = wg_reduce(ndef, Max32(), s_r32);
    if (ndef) {  // vertices the tiles could not hold, by the group scorer
      switch (in.lanes) {
        case 4: score_pass<4, T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, true, &evals2, &np2); break;
        case 8: score_pass<8, T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, true, &evals2, &np2); break;
        case 32: score_pass<32, T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, true, &evals2, &np2); break;
        case 64: score_pass<64, T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, true, &evals2, &np2); break;
        default: score_pass<16, T>(n, k, in.row_ptr, in.col, lit, C, Lvm, N.p, s, Ls, prop, dprop, true, &evals2, &np2); break;
      }
      __syncthreads();
    }
    evals = wg_reduce(evals + evals2, Add64(), s_r64);
    const int64_t nprop = wg_reduce((int64_t)np + np2, Add64(), s_r64);
    res.passes += 1;
    res.candidate_evals += evals;
    if (nprop == 0) {
      res.converged = 1;
      break;
    }
    // apply the whole batch, measuring the objective change
    int64_t dn2 = 0, ds2 = 0;
    apply_moves<T>(n, k, prop, C, Lvm, N, s, Ls, +1, 0, owner, dprop, &dn2, &ds2);
    dn2 = wg_reduce(dn2, Add64(), s_r64);
    ds2 = wg_reduce(ds2, Add64(), s_r64);
    const int64_t dO = (int64_t)k * ds2 - 2 * dn2;
    if (dO < 0) {
      O += dO;
      res.moves += nprop;
      for (int64_t v = t; v < n; v += kBlock)
        if (prop[v] >= 0) C[v] = prop[v];
    } else {
      res.fallback_rounds += 1;
      int64_t junk = 0;
      apply_moves<T>(n, k, prop, C, Lvm, N, s, Ls, -1, 0, owner, dprop, &junk, &junk);
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t to = prop[v];
        if (to < 0) continue;
        const uint64_t key = owner_key(dprop[v], v);
        atomicMin((unsigned long long*)&owner[C[v]], (unsigned long long)key);
        atomicMin((unsigned long long*)&owner[to], (unsigned long long)key);
      }
      __syncthreads();
      int64_t fn2 = 0, fs2 = 0;
      int64_t com = apply_moves<T>(n, k, prop, C, Lvm, N, s, Ls, +1, 1, owner, dprop, &fn2, &fs2);
      __syncthreads();
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t to = prop[v];
        if (to < 0) continue;
        const uint64_t key = owner_key(dprop[v], v);
        const bool own = owner[C[v]] == key && owner[to] == key;
        prop[v] = own ? to : -2 - to;
      }
      __syncthreads();
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t pv = prop[v];
        if (pv == kNone) continue;
        const int32_t to = pv >= 0 ? pv : -2 - pv;
        owner[C[v]] = ~0ull;
        owner[to] = ~0ull;
        if (pv >= 0) C[v] = pv;
      }
      fn2 = wg_reduce(fn2, Add64(), s_r64);
      fs2 = wg_reduce(fs2, Add64(), s_r64);
      com = wg_reduce(com, Add64(), s_r64);
      O += (int64_t)k * fs2 - 2 * fn2;
      res.moves += com;
    }
    __syncthreads();
    if (res.passes >= b.max_rounds) break;
  }
  // ---- output ----
  int64_t ncl = 0;
  for (int64_t v = t; v < n; v += kBlock) in.out[v] = rawid[C[v]];
  for (int64_t x = t; x < K0; x += kBlock) ncl += s[x] > 0;
  ncl = wg_reduce(ncl, Add64(), s_r64);
  res.clusters = (int32_t)ncl;
  res.objective = O;
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_batch(BatchArgs b) {
  __shared__ BatchLds L;
  __shared__ int32_t s_r32[kBlock / 64];
  __shared__ int64_t s_r64[kBlock / 64];
  __shared__ InstState S;
  __shared__ int32_t s_idx;
  const int t = threadIdx.x;
  // workspace slot of this workgroup
  const int64_t slot = blockIdx.x;
  const BatchWs& w = b.ws;
  int32_t* C = w.C + slot * w.n_max;
  int32_t* rawid = w.rawid + slot * w.n_max;
  int32_t* prop = w.prop + slot * w.n_max;
  int64_t* dprop = w.dprop + slot * w.n_max;
  int32_t* s = w.s + slot * w.n_max;
  uint64_t* owner = w.owner + slot * w.n_max;
  int32_t* Lvm = w.Lvm + slot * w.n_max * w.k_max;
  int32_t* N = w.N + slot * w.cells_cap;
  int32_t* flags = w.flags + slot * w.flag_cap;

  for (;;) {
    if (t == 0) s_idx = (int32_t)min(atomicAdd(b.queue, 1ull) - b.qbase, (unsigned long long)b.count);
    __syncthreads();
    const int32_t qi = __builtin_amdgcn_readfirstlane(s_idx);  // uniform: scalar loads below
    __syncthreads();
    if (qi >= b.count) break;
    const int32_t id = __builtin_amdgcn_readfirstlane(b.order[qi]);
    const BatchInst in = b.inst[id];
    BatchRes res = {};
    const int64_t t0 = wall_clock64();
    const int64_t n = in.n;
    const int32_t k = in.k;
    if (t == 0) {
      S.status = 0;
      S.acc = 0;
    }
    __syncthreads();
    // cluster ids must fit the tile scorer's 24-bit keys
    if (n > 0 && (n > w.n_max || k > w.k_max || n + 1 > w.flag_cap || n >= (1 << 24)))
      if (t == 0) S.status = kBatchTooBig;
    __syncthreads();
    if (n > 0 && !S.status) phase_clusters(n, k, in.init, flags, C, rawid, s, owner, L.su.h,
                                           s_r32, s_r64, &S);
    if (n > 0 && !S.status) phase_rows(n, k, in.labels, Lvm, s_r32, &S);
    if (n > 0 && !S.status) {
      res.cells = (int64_t)S.K0 * S.Ls * k;
      if (res.cells > w.cells_cap || (S.Ls > kLabLds && S.Ls > w.flag_cap)) {
        __syncthreads();
        if (t == 0) S.status = kBatchTooBig;
        __syncthreads();
      }
    }
    if (n > 0 && !S.status) {
      if (n < (1 << 15))
        run_instance<int16_t>(b, in, n, k, Counts<int16_t>{reinterpret_cast<int16_t*>(N)}, C,
                              rawid, prop, dprop, s, owner, Lvm, flags, L, s_r32, s_r64, &S, res);
      else
        run_instance<int32_t>(b, in, n, k, Counts<int32_t>{N}, C, rawid, prop, dprop, s, owner,
                              Lvm, flags, L, s_r32, s_r64, &S, res);
    }
    if (n == 0 || S.status) {
      if (t == 0) {
        res.status = S.status;
        if (n == 0) {
          res.passes = 1;
          res.converged = 1;
        }
        res.ticks = wall_clock64() - t0;
        b.res[id] = res;
      }
      __syncthreads();
      continue;
    }
    if (t == 0) {
      res.ticks = wall_clock64() - t0;
      b.res[id] = res;
    }
    __syncthreads();
  }
}

}  // namespace

bool batch_lanes_ok(int lanes) {
  return lanes == 0 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 || lanes == 64;
}

void launch_batch(const BatchArgs& a, int grid, hipStream_t st) {
  k_batch<<<grid, kBlock, 0, st>>>(a);
}

const void* batch_kernel() { return reinterpret_cast<const void*>(&k_batch); }

}  // namespace mcc
