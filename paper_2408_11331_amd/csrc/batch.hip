// Batched consensus: many independent instances in one persistent launch.
//
// Each workgroup pops an instance from a queue (largest estimated work
// first) and runs the whole method on it: consensus-cluster and label
// compaction, contingency tables, and the synchronous pass loop of the
// single-instance path (score every vertex against the frozen partition,
// apply the batch, keep it if the objective drops, else the conflict-free
// owner subset), with workgroup barriers in place of kernel boundaries.
// Per-instance state lives in a workspace slot owned by the workgroup for
// the duration of the instance.  An instance that exceeds a slot's
// capacities is reported back and solved by the single-instance path, so
// every output equals the single-instance output bit for bit.
#include "batch.h"

namespace mcc {

namespace {

constexpr int kBatchMaxK = 256;
constexpr int kBatchLds = 8192;  // int32 histogram entries in LDS (32 KiB)
constexpr int32_t kNone = -1;
constexpr int64_t kGainBias = (int64_t)1 << 33;

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

// In-place exclusive scan of a[0..len) by one workgroup; returns the total.
__device__ int32_t wg_scan(int32_t* a, int64_t len) {
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < len; b0 += kBlock) {
    const int64_t idx = b0 + threadIdx.x;
    const int32_t x = idx < len ? a[idx] : 0;
    int32_t tot;
    const int32_t e = block_exclusive_scan(x, &tot);
    if (idx < len) a[idx] = carry + e;
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// Apply (sign d) the move of v from `from` to `to` to sizes and counts;
// returns the change of the sums of squares (N part in *dn2, sizes in *ds2).
__device__ inline void bmove(int32_t* N, int32_t* s, const int32_t* Lvm, int32_t Lmax,
                             int32_t k, int64_t v, int32_t from, int32_t to, int32_t d,
                             int64_t* dn2, int64_t* ds2) {
  const int32_t* row = Lvm + v * k;
  for (int i = 0; i < k; ++i) {
    const int32_t l = row[i];
    const int32_t o1 = atomicAdd(&N[((int64_t)to * Lmax + l) * k + i], d);
    const int32_t o2 = atomicAdd(&N[((int64_t)from * Lmax + l) * k + i], -d);
    *dn2 += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
  }
  const int32_t o1 = atomicAdd(&s[to], d);
  const int32_t o2 = atomicAdd(&s[from], -d);
  *ds2 += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
}

// One scoring pass over the instance: G lanes per vertex, kBlock / G
// vertices at a time.  Candidates are taken in increasing cluster id by
// repeated group minima, so the result does not depend on G.  Kept out of
// line: inlined, the five variants share one register allocation and the
// kernel loses a wave per SIMD.
template <int G>
__device__ __attribute__((noinline)) void score_pass(const BatchInst& in, bool literal, const int32_t* C,
                           const int32_t* Lvm, const int32_t* N, const int32_t* s,
                           int32_t Lmax, int32_t* prop,
                           int64_t* dprop, int64_t* evals_out, int32_t* np_out) {
  constexpr int R = 8;  // arc registers per lane before re-reading memory
  constexpr int32_t kInf = 0x7fffffff;
  constexpr int NG = kBlock / G;
  const int lane = threadIdx.x & (G - 1), grp = threadIdx.x / G;
  const int64_t n = in.n;
  const int32_t k = in.k;
  int64_t evals = 0;
  int32_t np = 0;
  for (int64_t v = grp; v < n; v += NG) {
    const int32_t cv = C[v];
    const int64_t beg = in.row_ptr[v], end = in.row_ptr[v + 1];
    const bool fits = end - beg <= (int64_t)G * R;
    int32_t xr[R];
    if (fits) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t j = beg + r * G + lane;
        xr[r] = kInf;
        if (j < end) {
          const int32_t cu = C[in.col[j]];
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
          const int32_t cu = C[in.col[j]];
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

__global__ __launch_bounds__(kBlock) void k_batch(BatchArgs b) {
  __shared__ int32_t s_L[kBatchMaxK];
  __shared__ int32_t s_h[kBatchLds];  // label counts, then one table slice
  __shared__ int32_t s_r32[kBlock / 64];
  __shared__ int64_t s_r64[kBlock / 64];
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
    if (t == 0) s_idx = atomicAdd(b.queue, 1);
    __syncthreads();
    const int32_t qi = s_idx;
    __syncthreads();
    if (qi >= b.count) break;
    const int32_t id = b.order[qi];
    const BatchInst in = b.inst[id];
    BatchRes res = {};
    const int64_t t0 = wall_clock64();
    auto report = [&](BatchRes& r) {  // thread 0 only
      r.ticks = wall_clock64() - t0;
      b.res[id] = r;
    };
    const int64_t n = in.n;
    const int32_t k = in.k;
    if (n == 0) {
      if (t == 0) {
        res.passes = 1;
        res.converged = 1;
        report(res);
      }
      continue;
    }
    if (n > w.n_max || k > w.k_max || n + 1 > w.flag_cap) {
      if (t == 0) {
        res.status = kBatchTooBig;
        report(res);
      }
      continue;
    }
    // ---- consensus clusters: dense ids in order of the initial ids ----
    int32_t K0;
    if (in.init) {
      for (int64_t x = t; x <= n; x += kBlock) flags[x] = 0;
      __syncthreads();
      int32_t bad = 0;
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t x = in.init[v];
        if (x < 0 || x >= n) bad = 1;
        else flags[x] = 1;
      }
      bad = wg_reduce(bad, Max32(), s_r32);
      if (bad) {
        if (t == 0) {
          res.status = kBatchInvalid;
          report(res);
        }
        continue;
      }
      K0 = wg_scan(flags, n);
      if (t == 0) flags[n] = K0;
      __syncthreads();
      for (int64_t v = t; v < n; v += kBlock) {
        C[v] = flags[in.init[v]];
        if (flags[v + 1] > flags[v]) rawid[flags[v]] = (int32_t)v;
      }
    } else {
      K0 = (int32_t)n;
      for (int64_t v = t; v < n; v += kBlock) {
        C[v] = (int32_t)v;
        rawid[v] = (int32_t)v;
      }
    }
    __syncthreads();
    // ---- sizes, then labels and contingency table partition by partition ----
    // Each partition's label counts and its K0 x L_i slice of the table are
    // histogrammed in LDS when they fit and written once (no zero fill, no
    // global atomics); the objective's sums of squares come from the same
    // counts: O = k sum_x s_x^2 + sum_i sum_l |P_il|^2 - 2 sum N^2.
    const bool lds_sizes = K0 <= kBatchLds;
    for (int64_t x = t; x < K0; x += kBlock) {
      owner[x] = ~0ull;
      if (lds_sizes) s_h[x] = 0;
      else s[x] = 0;
    }
    __syncthreads();
    for (int64_t v = t; v < n; v += kBlock) {
      if (lds_sizes) atomicAdd(&s_h[C[v]], 1);
      else atomicAdd(&s[C[v]], 1);
    }
    __syncthreads();
    int64_t acc = 0;
    for (int64_t x = t; x < K0; x += kBlock) {
      const int32_t sx = lds_sizes ? s_h[x] : s[x];
      if (lds_sizes) s[x] = sx;
      acc += (int64_t)k * sx * sx;
    }
    __syncthreads();
    // labels: dense ids per partition (vertex-major rows) and |P_il|
    int32_t status = 0;
    int32_t Lmax = 1;  // same in every thread
    for (int i = 0; i < k; ++i) {
      const int32_t* p = in.labels[i];
      int32_t m = -1, lo = 0;
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t x = p[v];
        m = max(m, x);
        lo = min(lo, x);
      }
      m = wg_reduce(m, Max32(), s_r32);
      lo = wg_reduce(lo, Min32(), s_r32);
      if (lo < 0) {
        status = kBatchInvalid;
        break;
      }
      if ((int64_t)m + 2 > w.flag_cap) {
        status = kBatchTooBig;
        break;
      }
      // label sizes |P_il| (in LDS when the label values fit), then ids
      const bool lds_lab = (int64_t)m + 1 <= kBatchLds;
      for (int64_t x = t; x <= m; x += kBlock) {
        if (lds_lab) s_h[x] = 0;
        else flags[x] = 0;
      }
      __syncthreads();
      for (int64_t v = t; v < n; v += kBlock) {
        if (lds_lab) atomicAdd(&s_h[p[v]], 1);
        else atomicAdd(&flags[p[v]], 1);
      }
      __syncthreads();
      for (int64_t x = t; x <= m; x += kBlock) {
        const int32_t c = lds_lab ? s_h[x] : flags[x];
        acc += (int64_t)c * c;
        flags[x] = c > 0;
      }
      __syncthreads();
      const int32_t Li = wg_scan(flags, (int64_t)m + 1);  // flags: dense label ids
      if (t == 0) s_L[i] = Li;
      Lmax = max(Lmax, Li);
      for (int64_t v = t; v < n; v += kBlock) Lvm[v * k + i] = flags[p[v]];
      __syncthreads();
    }
    // interleaved table N[(x * Lmax + l) * k + i]: the k counts one probe of
    // a vertex needs lie side by side when its labels line up with its
    // cluster (any injective relabelling leaves the counts unchanged)
    const int64_t cells = (int64_t)K0 * Lmax * k;
    res.cells = cells;
    if (!status && cells > w.cells_cap) status = kBatchTooBig;
    if (status) {
      if (t == 0) {
        res.status = status;
        report(res);
      }
      __syncthreads();
      continue;
    }
    // one partition at a time: its K0 x L_i counts histogrammed in LDS when
    // they fit, written once; the sum of squares from the same counts
    for (int i = 0; i < k; ++i) {
      const int32_t Li = s_L[i];
      const int64_t entries = (int64_t)K0 * Li;
      const bool lds_tab = entries <= kBatchLds;
      for (int64_t j = t; j < entries; j += kBlock) {
        if (lds_tab) {
          s_h[j] = 0;
        } else {
          const int64_t x = j / Li;
          N[(x * Lmax + (j - x * Li)) * k + i] = 0;
        }
      }
      __syncthreads();
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t c = C[v], l = Lvm[v * k + i];
        if (lds_tab) atomicAdd(&s_h[(int64_t)c * Li + l], 1);
        else atomicAdd(&N[((int64_t)c * Lmax + l) * k + i], 1);
      }
      __syncthreads();
      for (int64_t j = t; j < entries; j += kBlock) {
        const int64_t x = j / Li;
        const int64_t cell = (x * Lmax + (j - x * Li)) * k + i;
        const int32_t c = lds_tab ? s_h[j] : N[cell];
        if (lds_tab) N[cell] = c;
        acc -= 2 * (int64_t)c * c;
      }
      __syncthreads();
    }
    int64_t O = wg_reduce(acc, Add64(), s_r64);
    res.objective_init = O;

    // ---- pass loop ----
    for (;;) {
      int64_t evals = 0;
      int32_t np = 0;
      const bool lit = b.literal != 0;
      switch (in.lanes) {
        case 4: score_pass<4>(in, lit, C, Lvm, N, s, Lmax, prop, dprop, &evals, &np); break;
        case 8: score_pass<8>(in, lit, C, Lvm, N, s, Lmax, prop, dprop, &evals, &np); break;
        case 32: score_pass<32>(in, lit, C, Lvm, N, s, Lmax, prop, dprop, &evals, &np); break;
        case 64: score_pass<64>(in, lit, C, Lvm, N, s, Lmax, prop, dprop, &evals, &np); break;
        default: score_pass<16>(in, lit, C, Lvm, N, s, Lmax, prop, dprop, &evals, &np); break;
      }
      evals = wg_reduce(evals, Add64(), s_r64);
      const int64_t nprop = wg_reduce((int64_t)np, Add64(), s_r64);
      res.passes += 1;
      res.candidate_evals += evals;
      if (nprop == 0) {
        res.converged = 1;
        break;
      }
      // apply the whole batch, measuring the objective change
      int64_t dn2 = 0, ds2 = 0;
      for (int64_t v = t; v < n; v += kBlock) {
        const int32_t to = prop[v];
        if (to >= 0) bmove(N, s, Lvm, Lmax, k, v, C[v], to, +1, &dn2, &ds2);
      }
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
        for (int64_t v = t; v < n; v += kBlock) {
          const int32_t to = prop[v];
          if (to < 0) continue;
          const int32_t from = C[v];
          bmove(N, s, Lvm, Lmax, k, v, from, to, -1, &junk, &junk);
          const uint64_t key = owner_key(dprop[v], v);
          atomicMin((unsigned long long*)&owner[from], (unsigned long long)key);
          atomicMin((unsigned long long*)&owner[to], (unsigned long long)key);
        }
        __syncthreads();
        int64_t fn2 = 0, fs2 = 0, com = 0;
        for (int64_t v = t; v < n; v += kBlock) {
          const int32_t to = prop[v];
          if (to < 0) continue;
          const int32_t from = C[v];
          const uint64_t key = owner_key(dprop[v], v);
          if (owner[from] == key && owner[to] == key) {
            bmove(N, s, Lvm, Lmax, k, v, from, to, +1, &fn2, &fs2);
            ++com;
          } else {
            prop[v] = -2 - to;
          }
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
    if (t == 0) report(res);
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

}  // namespace mcc
