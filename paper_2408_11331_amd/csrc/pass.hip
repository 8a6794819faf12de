// One synchronous pass of the greedy consensus (Methods, "Graph-aware
// consensus clustering" and "Parallel algorithm"):
//
//   score      every vertex, against the frozen partition, finds the
//              neighbour cluster with the smallest (gain, cluster id) and
//              proposes it when the gain is negative (Eq. objective3/4)
//   begin      count the pass; stop if nothing was proposed
//   apply      apply every proposal to sizes and counts, measuring the exact
//              change of the objective on the way
//   decide     keep the batch if the objective dropped, else fall back
//   commit     write the new cluster ids, or (fallback) undo the batch and
//              elect an owner per touched cluster
//   fb_commit  (fallback) apply the proposals that own both their clusters
//   fb_finish  (fallback) release owners, write the committed cluster ids
//   end        account the pass, enforce the pass cap
//
// Every kernel returns at once when the control block says the solve is
// done, so the host may enqueue passes ahead of the device.
//
// Gain of moving v from c to x (exact, the pair (v, v) left out):
//   2 (S_c(v) - S_x(v)) + k (s_x - s_c - 1),  S_y(v) = sum_i N_i(y, P_i(v)),
// obtained from Eq. objective3 by summing (k - 2 delta_uv) over the members
// of a cluster: delta_uv = k - #partitions agreeing on u, v, so the sum over
// y is 2 S_y(v) - k s_y.
//
// Objective bookkeeping: O = k sum_x s_x^2 + sum_i sum_l |P_i l|^2
// - 2 sum_i sum_(x,l) N_i(x,l)^2.  Each +-1 atomic update of a counter that
// returns the previous value `old` changes that counter's square by
// 2 old d + 1; summed over all updates of a pass this telescopes to the
// exact change of the sum of squares whatever order the atomics land in, so
// the batch's objective change is exact and deterministic.
#include "impl.h"

namespace mcc {

namespace {

constexpr int32_t kNone = -1;
constexpr int64_t kGainBias = (int64_t)1 << 33;

__device__ inline uint64_t owner_key(int64_t gain, int64_t v) {
  // (gain, vertex) ordered lexicographically; gain lies in (-2^33, 0) and
  // v in [0, 2^31)
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

// Exclusive prefix sum over the wave's lanes; *total: the wave's sum.
__device__ inline int32_t wave_excl_scan(int32_t x, int32_t* total) {
  const int lane = threadIdx.x & 63;
  int32_t s = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(s, o, 64);
    if (lane >= o) s += y;
  }
  *total = __shfl(s, 63, 64);
  return s - x;
}

__device__ inline int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ inline int32_t wave_sum32(int32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Add the workgroup's totals of the pass counters (all threads call; one
// atomic per counter and workgroup).
__device__ inline void flush_counts(const PassArgs& a, int64_t evals, int64_t nprop,
                                    int64_t boundary, int64_t skipped, int64_t wide = 0) {
  __shared__ int64_t red[kPassCounters][kBlock / 64];
  const int64_t v[kPassCounters] = {evals, nprop, boundary, skipped, wide};
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kPassCounters; ++c) {
    const int64_t x = wave_sum64(v[c]);
    if (lane == 0) red[c][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < kPassCounters) {
    int64_t tot = 0;
#pragma unroll
    for (int j = 0; j < kBlock / 64; ++j) tot += red[threadIdx.x][j];
    if (tot) atomicAdd((unsigned long long*)&a.pc[threadIdx.x * kCounterStride],
                       (unsigned long long)tot);
  }
}

// ---------------------------------------------------------------------------
// score: G lanes per vertex.  A lane keeps R neighbour cluster ids and the
// labels of up to KR partitions in registers; larger degrees or k fall back
// to re-reading memory.  Candidates are enumerated in increasing id by
// repeated group minima, so duplicates vanish and ties resolve to the
// smallest id without any sort.
// ---------------------------------------------------------------------------
constexpr int kMaxLdsPart = 256;  // partitions whose table geometry sits in LDS
constexpr int kTileCandAvg = 8;   // candidates per vertex the tiled scorer's key set holds
constexpr int kCandSetBits = 8;   // deferred vertex: LDS set of its candidate clusters
constexpr int kCandSet = 1 << kCandSetBits;

template <int G, bool LIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_score(PassArgs a) {
  if (a.ctl->done) return;
  // LIST: the vertices the tiled or list scorer deferred or, in a dense pass
  // the tiled scorer leaves to this kernel (defer_all), every vertex to
  // score: the rescoring list, or all vertices when there is none
  const bool all = LIST && a.ctl->defer_all && !(a.st && a.ctl->rescore_count <= a.sparse_max);
  const int64_t count =
      !LIST ? a.n : (all ? (a.st ? (int64_t)a.ctl->rescore_count : a.n) : (int64_t)a.ctl->heavy_count);
  if (LIST && count == 0) return;
  // arcs per lane held in registers; the deferred-vertex scorer (one wave
  // per vertex) holds 512, for the highest degrees
  constexpr int R = (LIST && G == 64) ? 8 : ((128 / G) < 16 ? ((128 / G) > 1 ? (128 / G) : 1) : 16);
  constexpr int KR = (64 / G) > 1 ? (64 / G) : 1;  // labels held per lane
  constexpr int32_t kInf = 0x7fffffff;
  __shared__ int64_t s_toff[kMaxLdsPart];
  __shared__ int32_t s_L[kMaxLdsPart];
  // deferred-vertex scorer, per wave: items' first member pair, sums, member
  // list starts, clusters, and the items of clusters without member lists
  constexpr int kW = (LIST && G == 64) ? kBlock / 64 : 1;
  constexpr int kI = (LIST && G == 64) ? 130 : 1;
  __shared__ int32_t s_ioff[kW][kI], s_isum[kW][kI], s_imst[kW][kI], s_iy[kW][kI],
      s_ilarge[kW][kI];
  __shared__ __align__(8) int32_t s_vrow[kW][(LIST && G == 64) ? 64 : 2];
  __shared__ int32_t s_cset[kW][(LIST && G == 64) ? kCandSet : 1];
  __shared__ int32_t s_cnb[kW][(LIST && G == 64) ? kCandSet : 1];  // a neighbour in the cluster
  __shared__ int32_t s_clist[kW][(LIST && G == 64) ? 128 : 1];
  __shared__ int32_t s_cnbl[kW][(LIST && G == 64) ? 128 : 1];
  __shared__ int32_t s_ccount[kW];
  const int lane = threadIdx.x & (G - 1);
  const int64_t group = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * kBlock) / G;
  const int32_t k = a.k;
  const bool kfits = k <= KR * G;
  for (int i = threadIdx.x; i < k && i < kMaxLdsPart; i += kBlock) {
    s_toff[i] = a.t.interleaved ? 0 : a.t.toff[i];  // no offsets when interleaved
    s_L[i] = a.t.L[i];
  }
  __syncthreads();
  const bool lds_geom = k <= kMaxLdsPart;

  int64_t evals = 0;
  int32_t nprop = 0, boundary = 0, wide = 0;
  for (int64_t idx = group; idx < count; idx += ngroups) {
    const int64_t v = !LIST ? idx : (all ? (a.st ? (int64_t)a.rlist[idx] : idx) : (int64_t)a.heavy[idx]);
    const int32_t cv = a.C[v];
    const int64_t beg = a.row_ptr[v], end = a.row_ptr[v + 1];
    const bool fits = end - beg <= (int64_t)G * R;
    int32_t x[R];
    if (fits) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t j = beg + r * G + lane;
        x[r] = kInf;
        if (j < end) {
          // a self-loop points at v's own cluster and drops out with it
          const int32_t cu = a.ac ? a.ac[j] : cn_load(a, a.col[j]);
          if (cu != cv) x[r] = cu;
        }
      }
    }
    // the label row is read only once the vertex has a candidate: interior
    // vertices (every neighbour in their own cluster) never touch it
    const int32_t* row = a.Lvm + v * k;
    int32_t lab[KR];
    bool have_row = false;
    auto load_row = [&]() {
      if (kfits && !have_row) {
#pragma unroll
        for (int t = 0; t < KR; ++t) {
          int i = lane + t * G;
          lab[t] = i < k ? row[i] : 0;
        }
      }
      have_row = true;
    };
    // S_y(v) summed over the group's lanes
    auto agree = [&](int32_t y) -> int32_t {
      int32_t sum = 0;
      if (a.members && a.s[y] <= a.msum_max) {
        // S_y(v) = sum over members u of y of the partitions agreeing on u, v;
        // the member ids are read once, one per lane, and broadcast
        const int32_t cnt = a.s[y], b = a.mstart[y];
        for (int32_t m0 = 0; m0 < cnt; m0 += G) {
          const int32_t mid = m0 + lane < cnt ? a.members[b + m0 + lane] : 0;
          const int32_t mc = min(G, cnt - m0);
          for (int32_t j = 0; j < mc; ++j) {
          const int32_t* ru = a.Lvm + (int64_t)__shfl(mid, j, G) * k;
          if (kfits) {
#pragma unroll
            for (int t = 0; t < KR; ++t) {
              int i = lane + t * G;
              if (i < k) sum += ru[i] == lab[t];
            }
          } else {
            for (int i = lane; i < k; i += G) sum += ru[i] == row[i];
          }
          }
        }
      } else if (a.t.hashed) {
        const uint64_t ky = (uint64_t)(uint32_t)y << 32;
        if (kfits && a.t.rows) {
#pragma unroll
          for (int t = 0; t < KR; ++t) {
            int i = lane + t * G;
            if (i < k) sum += hcount(a.t, i, y, lab[t]);
          }
        } else if (kfits) {  // implies lds_geom
#pragma unroll
          for (int t = 0; t < KR; ++t) {
            int i = lane + t * G;
            if (i < k) sum += hget(a.t, ky | (uint64_t)(s_toff[i] + lab[t]));
          }
        } else {
          for (int i = lane; i < k; i += G) sum += count_of(a.t, i, y, row[i]);
        }
      } else if (a.t.interleaved) {
        const int64_t base = (int64_t)y * a.t.Lmax;
        if (kfits) {
#pragma unroll
          for (int t = 0; t < KR; ++t) {
            int i = lane + t * G;
            if (i < k) sum += a.t.N[(base + lab[t]) * k + i];
          }
        } else {
          for (int i = lane; i < k; i += G) sum += a.t.N[(base + row[i]) * k + i];
        }
      } else if (kfits) {  // implies lds_geom
#pragma unroll
        for (int t = 0; t < KR; ++t) {
          int i = lane + t * G;
          if (i < k) sum += a.t.N[s_toff[i] + (int64_t)y * s_L[i] + lab[t]];
        }
      } else if (lds_geom) {
        for (int i = lane; i < k; i += G)
          sum += a.t.N[s_toff[i] + (int64_t)y * s_L[i] + row[i]];
      } else {
        for (int i = lane; i < k; i += G)
          sum += a.t.N[a.t.toff[i] + (int64_t)y * a.t.L[i] + row[i]];
      }
      return group_sum<G>(sum);
    };

    if constexpr (LIST && G == 64) {
      if (fits && kfits) {
        // a deferred vertex: its distinct candidate clusters collected in a
        // per-wave LDS hash set and compacted (lane j holds candidates j and
        // 64 + j, in no particular order: every argmin breaks ties by
        // cluster id), then its own cluster and the candidates scored, and
        // the smallest (gain, cluster id) taken by a wave reduction
        const int w = threadIdx.x >> 6;
        int32_t* cset = s_cset[w];
        int32_t* cnb = s_cnb[w];
        for (int j = lane; j < kCandSet; j += 64) cset[j] = -1;
        if (lane == 0) s_ccount[w] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int32_t y = x[r];
          if (y == kInf) continue;
          uint32_t h = ((uint32_t)y * 2654435761u) >> (32 - kCandSetBits);
          for (int q = 0; q < kCandSet; ++q) {  // bounded: a full set ends it
            int32_t cur = cset[h];
            if (cur == -1) {
              cur = atomicCAS(&cset[h], -1, y);
              if (cur == -1) {
                // the arc's head: a candidate of one vertex has it as its
                // only member
                cnb[h] = a.col[beg + r * 64 + lane];
                atomicAdd(&s_ccount[w], 1);
                break;
              }
            }
            if (cur == y) break;
            h = (h + 1) & (kCandSet - 1);
          }
        }
        __builtin_amdgcn_wave_barrier();
        int32_t nc = s_ccount[w];
        const bool many = nc > 128;  // more than 128 candidates: the general path below
        int32_t cand_lo = kInf, cand_hi = kInf;
        if (!many) {
          int32_t mine = 0, keys[kCandSet / 64];
#pragma unroll
          for (int q = 0; q < kCandSet / 64; ++q) {
            keys[q] = cset[lane + 64 * q];
            mine += keys[q] != -1;
          }
          int32_t total;
          int32_t pos = wave_excl_scan(mine, &total);
          int32_t* clist = s_clist[w];
          int32_t* cnbl = s_cnbl[w];
#pragma unroll
          for (int q = 0; q < kCandSet / 64; ++q)
            if (keys[q] != -1) {
              cnbl[pos] = cnb[lane + 64 * q];
              clist[pos++] = keys[q];
            }
          __builtin_amdgcn_wave_barrier();
          cand_lo = lane < nc ? clist[lane] : kInf;
          cand_hi = 64 + lane < nc ? clist[64 + lane] : kInf;
          __builtin_amdgcn_wave_barrier();
        }
        if (!many) {
          if (a.dirty) {  // the candidate set, cached for later passes
            if (lane < min(nc, kCacheCand)) a.ccache[v * kCacheCand + lane] = cand_lo;
            if (lane == 0) a.cnum[v] = nc <= kCacheCand ? nc : -1;
          }
          if (nc == 0) {
            if (lane == 0) a.prop[v] = kNone;
            continue;
          }
          const int sg = lane >> 4, sl = lane & 15;
          int32_t lb[4];  // labels of partitions sl + 16 q
#pragma unroll
          for (int q = 0; q < 4; ++q) lb[q] = sl + 16 * q < k ? row[sl + 16 * q] : 0;
          int32_t s_lo = 0, s_hi = 0, s_v = 0;
          const int nitems = nc + 1;  // item 0: the own cluster; item c + 1: candidate c
          if (a.members) {
            // Small clusters (member lists) are scored by their members' label
            // rows, every member row of every small item in flight at once:
            // four lanes per (item, member) pair, sixteen pairs a step, the
            // pair sums added into the item's LDS slot.  The other items
            // probe the table, one per 16-lane group.
            int32_t* ioff = s_ioff[w];
            int32_t* isum = s_isum[w];
            int32_t* imst = s_imst[w];
            int32_t* iy = s_iy[w];
            int32_t* ilarge = s_ilarge[w];
            // this lane's items: lane, 64 + lane and, for lane 0, 128
            const int32_t lo_prev = __shfl(cand_lo, (lane + 63) & 63, 64);
            const int32_t hi_prev = __shfl(cand_hi, (lane + 63) & 63, 64);
            const int32_t yA = lane == 0 ? cv : lo_prev;
            const int32_t yB = lane == 0 ? lo_prev : hi_prev;
            const int32_t yC = hi_prev;
            const bool vA = lane < nitems, vB = 64 + lane < nitems, vC = lane == 0 && 128 < nitems;
            // a member of each item: v for its own cluster, else the head of
            // an arc into the candidate (candidate c is item c + 1)
            const int32_t* cnbl = s_cnbl[w];
            const int32_t uA = lane == 0 ? (int32_t)v : (vA ? cnbl[lane - 1] : -1);
            const int32_t uB = vB ? cnbl[63 + lane] : -1;
            const int32_t uC = vC ? cnbl[127] : -1;
            const int32_t zA = vA ? a.s[yA] : 0, zB = vB ? a.s[yB] : 0, zC = vC ? a.s[yC] : 0;
            const bool smA = vA && zA <= a.msum_max, smB = vB && zB <= a.msum_max,
                       smC = vC && zC <= a.msum_max;
            // member list start, or ~u for a cluster whose one member u is known
            auto mlist = [&](bool sm, int32_t z, int32_t u, int32_t y) -> int32_t {
              return !sm ? 0 : ((z == 1 && u >= 0) ? ~u : a.mstart[y]);
            };
            const int32_t mA = mlist(smA, zA, uA, yA), mB = mlist(smB, zB, uB, yB),
                          mC = mlist(smC, zC, uC, yC);
            int32_t totA, totB, lgA, lgB;
            const int32_t exA = wave_excl_scan(smA ? zA : 0, &totA);
            const int32_t exB = wave_excl_scan(smB ? zB : 0, &totB);
            const int32_t gA = wave_excl_scan((vA && !smA) ? 1 : 0, &lgA);
            const int32_t gB = wave_excl_scan((vB && !smB) ? 1 : 0, &lgB);
            const int32_t cC = __shfl(smC ? zC : 0, 0, 64);
            const int32_t P = totA + totB + cC;  // member pairs
            ioff[lane] = exA;
            ioff[64 + lane] = totA + exB;
            isum[lane] = 0;
            isum[64 + lane] = 0;
            imst[lane] = mA;
            imst[64 + lane] = mB;
            iy[lane] = yA;
            iy[64 + lane] = yB;
            if (vA && !smA) ilarge[gA] = lane;
            if (vB && !smB) ilarge[lgA + gB] = 64 + lane;
            if (lane == 0) {
              ioff[128] = totA + totB;
              ioff[129] = P;
              isum[128] = 0;
              imst[128] = mC;
              iy[128] = yC;
              if (vC && !smC) ilarge[lgA + lgB] = 128;
            }
            const int32_t NL = lgA + lgB + __shfl((vC && !smC) ? 1 : 0, 0, 64);
            __builtin_amdgcn_wave_barrier();
            // the item of pair p: the last item whose first pair is at or
            // before p (items without pairs share their successor's offset)
            auto item_of = [&](int32_t p) {
              int lo = 0, hi = 128;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (ioff[mid] <= p) lo = mid;
                else hi = mid - 1;
              }
              return lo;
            };
            const int li = lane & 3, pq = lane >> 2;
            int32_t* vrow = s_vrow[w];  // the vertex's row, read by every pair
            vrow[lane] = lane < k ? row[lane] : 0;
            __builtin_amdgcn_wave_barrier();
            if ((k & 1) == 0) {  // rows 8-byte aligned: two partitions a load
              const int h = k >> 1;
              const int2* vl = reinterpret_cast<const int2*>(vrow);
              for (int32_t p0 = 0; p0 < P; p0 += 32) {
                int32_t sums[2], its[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                  const int32_t p = p0 + 16 * e + pq;
                  sums[e] = 0;
                  its[e] = -1;
                  if (p < P) {
                    const int it = item_of(p);
                    its[e] = it;
                    const int32_t ms = imst[it];
                    const int32_t u = ms < 0 ? ~ms : a.members[ms + (p - ioff[it])];
                    const int2* ru = reinterpret_cast<const int2*>(a.Lvm + (int64_t)u * k);
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                      if (li + 4 * t < h) {
                        const int2 q = ru[li + 4 * t], r = vl[li + 4 * t];
                        sums[e] += (q.x == r.x) + (q.y == r.y);
                      }
                  }
                }
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                  sums[e] += __shfl_xor(sums[e], 1, 4);
                  sums[e] += __shfl_xor(sums[e], 2, 4);
                  if (li == 0 && its[e] >= 0) atomicAdd(&isum[its[e]], sums[e]);
                }
              }
            } else {  // odd k: one partition a load
              for (int32_t p0 = 0; p0 < P; p0 += 16) {
                const int32_t p = p0 + pq;
                int32_t sum = 0, it = -1;
                if (p < P) {
                  it = item_of(p);
                  const int32_t ms = imst[it];
                  const int32_t u = ms < 0 ? ~ms : a.members[ms + (p - ioff[it])];
                  const int32_t* ru = a.Lvm + (int64_t)u * k;
#pragma unroll
                  for (int t = 0; t < 16; ++t)
                    if (li + 4 * t < k) sum += ru[li + 4 * t] == vrow[li + 4 * t];
                }
                sum += __shfl_xor(sum, 1, 4);
                sum += __shfl_xor(sum, 2, 4);
                if (li == 0 && it >= 0) atomicAdd(&isum[it], sum);
              }
            }
            // items of larger clusters: table probes, four items a step
            for (int32_t j0 = 0; j0 < NL; j0 += 4) {
              const int32_t jj = j0 + sg;
              int32_t sum = 0, it = -1;
              if (jj < NL) {
                it = ilarge[jj];
                const int32_t y = iy[it];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                  if (sl + 16 * q < k) sum += count_of(a.t, sl + 16 * q, y, lb[q]);
              }
              sum = group_sum<16>(sum);
              if (sl == 0 && it >= 0) isum[it] = sum;
            }
            __builtin_amdgcn_wave_barrier();
            s_v = isum[0];
            s_lo = isum[1 + lane];
            s_hi = lane < 64 ? isum[65 + lane] : 0;
            __builtin_amdgcn_wave_barrier();
          } else {
            for (int j0 = 0; j0 < nitems; j0 += 4) {
              const int it = j0 + sg, ci = it - 1;
              const int32_t y_lo = __shfl(cand_lo, ci < 0 ? 0 : (ci & 63), 64);
              const int32_t y_hi = __shfl(cand_hi, ci < 0 ? 0 : (ci & 63), 64);
              const int32_t y = it == 0 ? cv : (ci < 64 ? y_lo : y_hi);
              int32_t sum = 0;
              if (it < nitems) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                  if (sl + 16 * q < k) sum += count_of(a.t, sl + 16 * q, y, lb[q]);
              }
              sum = group_sum<16>(sum);
              if (j0 == 0) s_v = __shfl(sum, 0, 64);
              const int g_lo = lane + 1 - j0, g_hi = lane + 65 - j0;  // groups holding my items
              const int32_t got_lo = __shfl(sum, (g_lo >= 0 && g_lo < 4) ? g_lo * 16 : 0, 64);
              const int32_t got_hi = __shfl(sum, (g_hi >= 0 && g_hi < 4) ? g_hi * 16 : 0, 64);
              if (g_lo >= 0 && g_lo < 4) s_lo = got_lo;
              if (g_hi >= 0 && g_hi < 4) s_hi = got_hi;
            }
          }
          const int64_t scv = a.s[cv];
          int64_t bd = INT64_MAX;
          int32_t bx = kInf;
          auto consider = [&](int32_t xc, int32_t sx) {
            int64_t d = 2 * ((int64_t)s_v - sx) + (int64_t)k * ((int64_t)a.s[xc] - scv - 1);
            if (a.literal) d += k;
            if (d < bd || (d == bd && xc < bx)) {
              bd = d;
              bx = xc;
            }
          };
          if (lane < nc) consider(cand_lo, s_lo);
          if (lane + 64 < nc) consider(cand_hi, s_hi);
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            const int64_t od = __shfl_xor(bd, o, 64);
            const int32_t ox = __shfl_xor(bx, o, 64);
            if (od < bd || (od == bd && ox < bx)) {
              bd = od;
              bx = ox;
            }
          }
          if (lane == 0) {
            evals += nc;
            boundary += 1;
            wide += nc > kTileCandAvg;
            const bool p = bd < 0;
            a.prop[v] = p ? bx : kNone;
            if (p) {
              a.dprop[v] = bd;
              ++nprop;
            }
            if (a.slack) a.slack[v] = p ? -1 : (int32_t)min(bd, (int64_t)INT32_MAX);
          }
          continue;
        }
        // the arc registers again, for the general path
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t j = beg + r * G + lane;
          x[r] = kInf;
          if (j < end) {
            const int32_t cu = a.ac ? a.ac[j] : cn_load(a, a.col[j]);
            if (cu != cv) x[r] = cu;
          }
        }
        if (a.dirty && lane == 0) a.cnum[v] = -1;
      }
    }

    int32_t last = -1, ncand = 0, bestx = kNone;
    int64_t bestd = 0, s_own = -1;
    const int64_t sc = a.s[cv];
    for (;;) {
      int32_t m = kInf;
      if (fits) {
#pragma unroll
        for (int r = 0; r < R; ++r) m = min(m, x[r]);
      } else {
        for (int64_t j = beg + lane; j < end; j += G) {
          const int32_t cu = a.ac ? a.ac[j] : cn_load(a, a.col[j]);
          if (cu != cv && cu > last && cu < m) m = cu;
        }
      }
      m = group_min<G>(m);
      if (m == kInf) break;
      if (s_own < 0) {
        load_row();
        s_own = agree(cv);
      }
      const int64_t sx = agree(m);
      int64_t d = 2 * (s_own - sx) + (int64_t)k * ((int64_t)a.s[m] - sc - 1);
      if (a.literal) d += k;
      if (ncand == 0 || d < bestd) {
        bestd = d;
        bestx = m;
      }
      ++ncand;
      last = m;
      if (fits) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (x[r] == m) x[r] = kInf;
      }
    }
    if (lane == 0) {
      evals += ncand;
      boundary += ncand > 0;
      wide += ncand > kTileCandAvg;
      const bool p = ncand > 0 && bestd < 0;
      a.prop[v] = p ? bestx : kNone;
      if (p) {
        a.dprop[v] = bestd;
        ++nprop;
      }
    }
  }
  flush_counts(a, evals, nprop, boundary, 0, wide);
}

// ---------------------------------------------------------------------------
// Tiled scorer.  A workgroup owns a tile of kBlock consecutive vertices:
//  1. the tile's row offsets and clusters go to LDS;
//  2. its arcs are walked in chunks, every thread taking consecutive arcs
//     with independent loads; each arc whose head lies in another cluster
//     inserts the key (tail, head cluster) into a tile-wide LDS hash set and
//     the first insertion of a key counts a candidate for the tail (a
//     self-loop points at the own cluster and drops out with it);
//  3. the set is compacted into one run of pairs per boundary vertex, its
//     own cluster first, then its candidate clusters;
//  4. groups of kProbeLanes lanes probe the flat list of pairs, lanes spread
//     over the partitions, with the next batch's label rows in flight while
//     the current batch probes (consecutive pairs of one vertex share one
//     load of its label row);
//  5. one thread per vertex takes the smallest (gain, cluster id).
// A vertex whose key finds no slot in the set is deferred to a list that
// the group scorer finishes in the same pass, so results never depend on
// the set's capacity.
// ---------------------------------------------------------------------------
constexpr int kArcChunk = 1024;
constexpr int kSetSlots = 2048;
constexpr int kSetProbe = 64;
constexpr int kPairMax = kSetSlots + kBlock;  // every candidate plus one own pair per vertex
constexpr int kProbeLanes = 16;
constexpr int kProbeRegs = 64 / kProbeLanes;  // labels per lane when k <= 64
constexpr int kProbeBatch = 4;
static_assert(kMemberSumMax <= kProbeLanes, "member ids of a small cluster fit one probe group");
static_assert(kSetSlots / kBlock == kTileCandAvg, "the tile's key set per vertex");

template <int CN, int TK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_score_tile(PassArgs a) {
  if (a.ctl->done) return;
  __shared__ int32_t s_off[kBlock + 1];
  __shared__ int32_t s_c[kBlock];
  __shared__ int32_t s_nc[kBlock];    // candidates of each vertex
  __shared__ int32_t s_def[kBlock];   // 1: vertex deferred to the group scorer
  __shared__ int32_t s_cur[kBlock];   // fill cursor of the vertex's run
  __shared__ int32_t s_clean[kBlock]; // 1: candidate set taken from the cache
  __shared__ int32_t s_np;            // pairs that fit the pair arrays
  __shared__ int32_t s_set[kSetSlots];
  __shared__ int32_t s_cl[kPairMax];   // pair keys (vertex << 24 | cluster), run per vertex
  __shared__ int32_t s_S[kPairMax];    // agreement sum of each pair
  const int t = threadIdx.x;
  const int32_t k = a.k;
  const bool kfits = k <= kProbeRegs * kProbeLanes;
  const int g = t / kProbeLanes, lane = t % kProbeLanes;
  int64_t evals = 0;
  int32_t nprop = 0, boundary = 0, wide = 0;
  const int64_t ntiles = (a.n + kBlock - 1) / kBlock;
  // passes with few vertices to rescore are left to the list scorer, and
  // passes whose vertices mostly have more candidates than a tile holds to
  // the wave-per-vertex scorer
  if (a.st && a.ctl->rescore_count <= a.sparse_max) return;
  if (a.ctl->defer_all) return;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t v0 = tile * kBlock;
    const int nv = (int)min((int64_t)kBlock, a.n - v0);
    const int32_t cv = t < nv ? a.C[v0 + t] : -1;
    s_c[t] = cv;
    // candidates of a vertex that need not be found again (from the status
    // pass: 0 also for a vertex already settled), -1: walk its arcs
    int32_t cached = -1;
    if (a.st && t < nv) {
      const int32_t stv = a.st[v0 + t];
      cached = stv < 0 ? 0 : (stv > 0 ? stv : -1);
    }
    s_clean[t] = cached >= 0;
    s_nc[t] = cached > 0 ? cached : 0;
    s_def[t] = 0;
    for (int j = t; j < kSetSlots; j += kBlock) s_set[j] = -1;
    // the arcs are walked only when some vertex of the tile needs them
    const int walk = __syncthreads_or(t < nv && cached < 0);
    int64_t a0 = 0;
    if (walk) {
      a0 = a.row_ptr[v0];
      for (int j = t; j <= nv; j += kBlock) s_off[j] = (int32_t)(a.row_ptr[v0 + j] - a0);
    } else if (t == 0) {
      s_off[nv] = 0;
    }
    __syncthreads();
    const int32_t A = s_off[nv];
    // each thread takes U consecutive arcs of every chunk, read as one
    // 16-byte load from an aligned arc index (the tile's arcs are walked from
    // the aligned index at or before its first arc): one search for the tail
    // of the first, then a walk along the row offsets
    constexpr int U = kArcChunk / kBlock;
    static_assert(U == 4, "one int4 load per thread and chunk");
    const int32_t sh = a.arcs_aligned ? (int32_t)(a0 & 3) : 0;
    const int64_t base = a0 - sh;
    const int32_t* src = CN ? a.col : a.ac;  // heads, or the per-arc clusters
    for (int32_t cb = 0; cb < A + sh; cb += kArcChunk) {
      const int32_t jt = cb + t * U - sh;  // tile-relative index of the thread's first arc
      int32_t hd[U];
      if (jt + U > 0 && jt < A) {
        const int64_t gi = base + cb + t * U;
        if (a.arcs_aligned && gi + U <= a.nnz) {
          const int4 q4 = *reinterpret_cast<const int4*>(src + gi);
          hd[0] = q4.x;
          hd[1] = q4.y;
          hd[2] = q4.z;
          hd[3] = q4.w;
        } else {
#pragma unroll
          for (int r = 0; r < U; ++r) {
            const int32_t j = jt + r;
            hd[r] = (j >= 0 && j < A) ? src[a0 + j] : 0;
          }
        }
      }
      int lo = 0;
      const int32_t j0 = max(jt, 0);
      if (j0 < A) {
        int hi = nv - 1;  // tail: the last vertex whose row starts at or before j0
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= j0) lo = mid;
          else hi = mid - 1;
        }
      }
      // tails of the thread's arcs; clean tails skip the gather
      int tl[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int32_t j = jt + r;
        tl[r] = -1;
        if (j < 0 || j >= A) continue;
        while (s_off[lo + 1] <= j) ++lo;
        if (!s_clean[lo]) tl[r] = lo;
      }
      int32_t cu[U];
#pragma unroll
      for (int r = 0; r < U; ++r) cu[r] = tl[r] >= 0 ? (CN ? cn_load_t<CN>(a, 0, hd[r]) : hd[r]) : -1;
      int32_t prev = -1;  // the last key this thread placed: repeats skip the set
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (tl[r] < 0) continue;
        lo = tl[r];
        const int32_t x = cu[r];
        if (x == s_c[lo] || s_def[lo]) continue;  // a deferred vertex needs no more keys
        const int32_t key = (lo << 24) | x;
        if (key == prev) continue;
        prev = key;
        uint32_t h = ((uint32_t)key * 2654435761u) >> 21;  // 11 bits: kSetSlots
        bool placed = false;
        for (int q = 0; q < kSetProbe; ++q) {
          int32_t cur = s_set[h];
          if (cur == -1) cur = atomicCAS(&s_set[h], -1, key);
          if (cur == -1) {  // first sighting of (lo, x)
            atomicAdd(&s_nc[lo], 1);
            placed = true;
            break;
          }
          if (cur == key) {
            placed = true;
            break;
          }
          h = (h + 1) & (kSetSlots - 1);
        }
        if (!placed) s_def[lo] = 1;
      }
    }
    __syncthreads();
    const int nc = s_nc[t];
    bool def = t < nv && s_def[t];
    bool is_b = t < nv && nc > 0 && !def;
    // one run per boundary vertex: its own cluster, then its candidates.
    // Candidates taken from the key set number at most kSetSlots, but cached
    // sets bypass it: a run that would pass the end of the pair arrays
    // defers its vertex (and the runs after it) to the group scorer.
    int32_t npairs;
    const int32_t coff = block_exclusive_scan(is_b ? nc + 1 : 0, &npairs);
    if (t == 0) s_np = npairs;
    __syncthreads();
    if (is_b && coff + nc + 1 > kPairMax) {
      is_b = false;
      def = true;
      s_def[t] = 1;
      atomicMin(&s_np, coff);
    }
    if (t < nv) {
      const int64_t v = v0 + t;
      if (def) {
        const int32_t slot = atomicAdd(&a.ctl->heavy_count, 1);
        a.heavy[slot] = (int32_t)v;
        if (a.slack) a.slack[v] = -1;
      } else if (nc == 0) {
        a.prop[v] = kNone;
      } else {
        evals += nc;
        boundary += 1;
        wide += nc > kTileCandAvg;
      }
    }
    s_cur[t] = coff + 1;
    if (is_b) {
      s_cl[coff] = (t << 24) | s_c[t];
      if (s_clean[t])
        for (int j = 0; j < nc; ++j)
          s_cl[coff + 1 + j] = (t << 24) | a.ccache[(v0 + t) * kCacheCand + j];
    }
    __syncthreads();
    npairs = s_np;
    for (int h = t; h < kSetSlots; h += kBlock) {
      const int32_t key = s_set[h];
      if (key == -1) continue;
      const int tv = (int)((uint32_t)key >> 24);
      if (s_def[tv]) continue;
      s_cl[atomicAdd(&s_cur[tv], 1)] = key;
    }
    __syncthreads();
    // cache the sets found this pass (interior vertices cache "none")
    if (a.dirty && t < nv && !s_clean[t]) {
      const int64_t v = v0 + t;
      if (def || nc > kCacheCand) {
        a.cnum[v] = -1;
      } else {
        for (int j = 0; j < nc; ++j) a.ccache[v * kCacheCand + j] = s_cl[coff + 1 + j] & 0xffffff;
        a.cnum[v] = nc;
      }
    }
    constexpr int kStride = (kBlock / kProbeLanes) * kProbeBatch;
    auto pair_at = [&](int p, int32_t& x, uint32_t& row) {
      x = -1;
      row = 0;
      if (p < npairs) {
        const int32_t key = s_cl[p];
        x = key & 0xffffff;
        row = (uint32_t)(v0 + (int)((uint32_t)key >> 24)) * (uint32_t)k;
      }
    };
    // label rows of a batch; a pair of the same vertex as the one before it
    // takes that pair's registers instead of loading again
    auto load_rows = [&](const int32_t* xq, const uint32_t* vq, int32_t (*lq)[kProbeRegs]) {
#pragma unroll
      for (int q = 0; q < kProbeBatch; ++q) {
        const bool same = q > 0 && xq[q - 1] >= 0 && vq[q] == vq[q - 1];
#pragma unroll
        for (int r = 0; r < kProbeRegs; ++r) {
          const int i = lane + r * kProbeLanes;
          lq[q][r] = (xq[q] >= 0 && i < k && !same) ? a.Lvm[vq[q] + i] : 0;
        }
      }
#pragma unroll
      for (int q = 1; q < kProbeBatch; ++q)
        if (xq[q - 1] >= 0 && vq[q] == vq[q - 1]) {
#pragma unroll
          for (int r = 0; r < kProbeRegs; ++r) lq[q][r] = lq[q - 1][r];
        }
    };
    if (kfits) {
      int32_t xs[kProbeBatch], lab[kProbeBatch][kProbeRegs];
      uint32_t vs[kProbeBatch];
      int p0 = g * kProbeBatch;
#pragma unroll
      for (int q = 0; q < kProbeBatch; ++q) pair_at(p0 + q, xs[q], vs[q]);
      load_rows(xs, vs, lab);
      for (; p0 < npairs; p0 += kStride) {
        int32_t xn[kProbeBatch], labn[kProbeBatch][kProbeRegs];
        uint32_t vn[kProbeBatch];
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) pair_at(p0 + kStride + q, xn[q], vn[q]);
        load_rows(xn, vn, labn);
        int32_t sums[kProbeBatch];
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          int32_t sum = 0;
          if (TK == kHashed && xs[q] >= 0 && a.members && a.s[xs[q]] <= a.msum_max) {
            const int32_t cnt = a.s[xs[q]];  // <= kProbeLanes: one member id per lane
            const int32_t mid = lane < cnt ? a.members[a.mstart[xs[q]] + lane] : 0;
            for (int32_t m = 0; m < cnt; ++m) {
              const uint32_t ru = (uint32_t)__shfl(mid, m, kProbeLanes) * (uint32_t)k;
#pragma unroll
              for (int r = 0; r < kProbeRegs; ++r) {
                const int i = lane + r * kProbeLanes;
                if (i < k) sum += a.Lvm[ru + i] == lab[q][r];
              }
            }
          } else {
#pragma unroll
            for (int r = 0; r < kProbeRegs; ++r) {
              const int i = lane + r * kProbeLanes;
              if (xs[q] >= 0 && i < k) sum += count_t<TK>(a.t, i, xs[q], lab[q][r]);
            }
          }
          sums[q] = sum;
        }
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          const int32_t sq = group_sum<kProbeLanes>(sums[q]);
          if (lane == 0 && xs[q] >= 0) s_S[p0 + q] = sq;
        }
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          xs[q] = xn[q];
          vs[q] = vn[q];
#pragma unroll
          for (int r = 0; r < kProbeRegs; ++r) lab[q][r] = labn[q][r];
        }
      }
    } else {
      for (int p0 = g * kProbeBatch; p0 < npairs; p0 += kStride) {
#pragma unroll
        for (int q = 0; q < kProbeBatch; ++q) {
          int32_t x;
          uint32_t ro;
          pair_at(p0 + q, x, ro);
          int32_t sum = 0;
          if (x >= 0) {
            const int32_t* row = a.Lvm + ro;
            if (TK == kHashed && a.members && a.s[x] <= a.msum_max) {
              const int32_t cnt = a.s[x];
              const int32_t mid = lane < cnt ? a.members[a.mstart[x] + lane] : 0;
              for (int32_t m = 0; m < cnt; ++m) {
                const int32_t* ru = a.Lvm + (int64_t)__shfl(mid, m, kProbeLanes) * k;
                for (int i = lane; i < k; i += kProbeLanes) sum += ru[i] == row[i];
              }
            } else {
              for (int i = lane; i < k; i += kProbeLanes) sum += count_t<TK>(a.t, i, x, row[i]);
            }
          }
          const int32_t sq = group_sum<kProbeLanes>(sum);
          if (lane == 0 && x >= 0) s_S[p0 + q] = sq;
        }
      }
    }
    __syncthreads();
    if (is_b) {
      const int64_t v = v0 + t;
      const int32_t c = s_c[t];
      const int64_t s_own = s_S[coff];
      const int64_t scz = a.s[c];
      int64_t bestd = 0;
      int32_t bestx = kNone;
      for (int j = coff + 1; j <= coff + nc; ++j) {
        const int32_t x = s_cl[j] & 0xffffff;
        int64_t d = 2 * (s_own - (int64_t)s_S[j]) + (int64_t)k * ((int64_t)a.s[x] - scz - 1);
        if (a.literal) d += k;
        if (bestx == kNone || d < bestd || (d == bestd && x < bestx)) {
          bestd = d;
          bestx = x;
        }
      }
      const bool p = bestd < 0;
      a.prop[v] = p ? bestx : kNone;
      if (p) {
        a.dprop[v] = bestd;
        ++nprop;
      }
      if (a.slack) a.slack[v] = p ? -1 : (int32_t)min(bestd, (int64_t)INT32_MAX);
    }
    __syncthreads();
  }
  flush_counts(a, evals, nprop, boundary, 0, wide);
}

// ---------------------------------------------------------------------------
// Status of every vertex at the start of a pass (with the candidate cache),
// one thread per vertex.  A vertex is settled here when it has no candidate
// (a clean vertex whose cached set is empty) or when the bound on the
// change of its gains since its last exact scoring cannot make any of them
// negative (it would not propose: its decision is written and its
// candidates counted as scored, as the method scores them).  Every other
// vertex goes to the rescoring list.  Also clears this pass's dirty marks
// and the per-cluster move counts the coming apply fills.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_status(PassArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  __shared__ int32_t s_base;
  const int par = ctl->passes & 1;
  const int32_t* churn = a.churn + (int64_t)par * a.K0;
  int32_t* next = a.churn + (int64_t)(par ^ 1) * a.K0;
  const int t = threadIdx.x;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + t; x < a.K0; x += (int64_t)gridDim.x * kBlock)
    next[x] = 0;
  const int32_t k = a.k;
  constexpr int V = 4;  // vertices per thread and chunk: v = c0 + j kBlock + t
  constexpr int64_t kChunk = (int64_t)V * kBlock;
  int64_t evals = 0, skipped = 0, boundary = 0;
  for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < a.n; c0 += (int64_t)gridDim.x * kChunk) {
    int32_t d[V], cn[V], sl[V], cv[V], stv[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t v = c0 + j * kBlock + t;
      d[j] = 1;
      cn[j] = -1;
      sl[j] = -1;
      cv[j] = 0;
      if (v < a.n) {
        d[j] = a.dirty[v];
        cn[j] = a.cnum[v];
        sl[j] = a.slack[v];
        cv[j] = a.C[v];
      }
    }
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t v = c0 + j * kBlock + t;
      stv[j] = -1;
      if (v >= a.n) continue;
      if (d[j]) a.dirty[v] = 0;  // this pass's moves mark it again
      const int32_t cached = d[j] ? -1 : cn[j];
      if (cached == 0) {
        a.prop[v] = kNone;
      } else if (cached > 0) {
        stv[j] = cached;
        if (sl[j] >= 0) {
          const int4* cc = reinterpret_cast<const int4*>(a.ccache + v * kCacheCand);
          const int4 c_lo = cc[0], c_hi = cached > 4 ? cc[1] : make_int4(0, 0, 0, 0);
          const int32_t ids[kCacheCand] = {c_lo.x, c_lo.y, c_lo.z, c_lo.w,
                                           c_hi.x, c_hi.y, c_hi.z, c_hi.w};
          int32_t mx = 0;
#pragma unroll
          for (int q = 0; q < kCacheCand; ++q)
            if (q < cached) mx = max(mx, churn[ids[q]]);
          const int64_t bound = (int64_t)k * ((int64_t)churn[cv[j]] + mx);
          if ((int64_t)sl[j] >= bound) {  // no candidate's gain can have become negative
            a.slack[v] = (int32_t)(sl[j] - bound);
            a.prop[v] = kNone;
            evals += cached;
            skipped += cached;
            boundary += 1;
            stv[j] = -1;
          }
        }
      } else {
        stv[j] = 0;
      }
      a.st[v] = stv[j];
      mine += stv[j] >= 0;
    }
    // the chunk's vertices left for scoring, appended with one atomic
    int32_t total;
    int32_t off = block_exclusive_scan(mine, &total);
    if (t == 0 && total) s_base = atomicAdd(&ctl->rescore_count, total);
    __syncthreads();
    if (total) {
      off += s_base;
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (stv[j] >= 0) a.rlist[off++] = (int32_t)(c0 + j * kBlock + t);
    }
    __syncthreads();
  }
  flush_counts(a, evals, 0, boundary, skipped);
}

// ---------------------------------------------------------------------------
// List scorer: the vertices of the rescoring list, in passes where they are
// few, kListLanes lanes per vertex.  A vertex's candidates come from its
// cache or from its arcs (distinct neighbour clusters, in increasing id, one
// per lane); its own cluster and the candidates are then probed four at a
// time with every probe of the four issued together.  Vertices with more
// candidates than lanes, a degree beyond the arc registers or k beyond the
// label registers go to the deferred list (the wave-per-vertex scorer).
// ---------------------------------------------------------------------------
constexpr int kListLanes = 16;

template <int CN, int TK>
__global__ __launch_bounds__(kBlock) void k_score_list(PassArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  const int32_t count = ctl->rescore_count;
  if (count == 0 || count > a.sparse_max) return;  // the tiled scorer takes dense passes
  constexpr int G = kListLanes;
  constexpr int R = 8;               // arcs per lane in registers: degree <= 128
  constexpr int KR = 64 / G;         // labels per lane: k <= 64
  constexpr int32_t kInf = 0x7fffffff;
  const int lane = threadIdx.x & (G - 1);
  const int64_t group = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int64_t ngroups = ((int64_t)gridDim.x * kBlock) / G;
  const int32_t k = a.k;
  int64_t evals = 0;
  int32_t nprop = 0, boundary = 0, wide = 0;
  for (int64_t idx = group; idx < count; idx += ngroups) {
    const int64_t v = a.rlist[idx];
    const int32_t cv = a.C[v];
    const int32_t stv = a.st[v];
    int32_t cand = kInf, nc = 0;
    bool defer = k > KR * G;
    if (!defer && stv > 0) {
      nc = stv;
      if (lane < nc) cand = a.ccache[v * kCacheCand + lane];
    } else if (!defer) {
      const int64_t beg = a.row_ptr[v], end = a.row_ptr[v + 1];
      if (end - beg > (int64_t)G * R) {
        defer = true;
      } else {
        int32_t x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t j = beg + r * G + lane;
          x[r] = kInf;
          if (j < end) {
            const int32_t cu = cn_load_t<CN>(a, j, CN ? a.col[j] : 0);
            if (cu != cv) x[r] = cu;
          }
        }
        for (;;) {  // distinct clusters in increasing id, candidate j on lane j
          int32_t m = kInf;
#pragma unroll
          for (int r = 0; r < R; ++r) m = min(m, x[r]);
          m = group_min<G>(m);
          if (m == kInf) break;
          if (nc == G) {
            defer = true;
            break;
          }
          if (lane == nc) cand = m;
          ++nc;
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (x[r] == m) x[r] = kInf;
        }
        if (!defer) {  // the set found, cached for later passes
          if (lane < min(nc, kCacheCand)) a.ccache[v * kCacheCand + lane] = cand;
          if (lane == 0) a.cnum[v] = nc <= kCacheCand ? nc : -1;
        }
      }
    }
    if (defer) {
      if (lane == 0) {
        a.heavy[atomicAdd(&ctl->heavy_count, 1)] = (int32_t)v;
        a.cnum[v] = -1;
        a.slack[v] = -1;
      }
      continue;
    }
    if (nc == 0) {
      if (lane == 0) {
        a.prop[v] = kNone;
        a.slack[v] = -1;
      }
      continue;
    }
    int32_t lab[KR];
    const int32_t* row = a.Lvm + v * k;
#pragma unroll
    for (int t = 0; t < KR; ++t) {
      const int i = lane + t * G;
      lab[t] = i < k ? row[i] : 0;
    }
    const int64_t scv = a.s[cv];
    int64_t s_own = 0, bd = 0;
    int32_t bx = kNone;
    for (int i0 = 0; i0 <= nc; i0 += 4) {  // item 0: own cluster; item j: candidate j - 1
      int32_t part[4], ys[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int it = i0 + q;
        const int32_t yc = __shfl(cand, it > 0 ? (it - 1) & (G - 1) : 0, G);
        ys[q] = it == 0 ? cv : (it <= nc ? yc : -1);
        part[q] = 0;
        if (ys[q] >= 0) {
#pragma unroll
          for (int t = 0; t < KR; ++t) {
            const int i = lane + t * G;
            if (i < k) part[q] += count_t<TK>(a.t, i, ys[q], lab[t]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t sum = group_sum<G>(part[q]);
        if (ys[q] < 0) continue;
        if (i0 + q == 0) {
          s_own = sum;
          continue;
        }
        int64_t d = 2 * (s_own - sum) + (int64_t)k * ((int64_t)a.s[ys[q]] - scv - 1);
        if (a.literal) d += k;
        if (bx == kNone || d < bd || (d == bd && ys[q] < bx)) {
          bd = d;
          bx = ys[q];
        }
      }
    }
    if (lane == 0) {
      evals += nc;
      boundary += 1;
      wide += nc > kTileCandAvg;
      const bool p = bd < 0;
      a.prop[v] = p ? bx : kNone;
      if (p) {
        a.dprop[v] = bd;
        ++nprop;
      }
      a.slack[v] = p ? -1 : (int32_t)min(bd, (int64_t)INT32_MAX);
    }
  }
  flush_counts(a, evals, nprop, boundary, 0, wide);
}

__global__ void k_begin(Ctl* ctl, int64_t* pc) {
  if (ctl->done) return;
  int64_t c[kPassCounters];
#pragma unroll
  for (int j = 0; j < kPassCounters; ++j) {
    c[j] = pc[j * kCounterStride];
    pc[j * kCounterStride] = 0;
  }
  ctl->pass_evals = c[0];
  ctl->nprop = (int32_t)c[1];
  ctl->boundary += c[2];
  ctl->skipped += c[3];
  // most boundary vertices had more candidates than the tiles hold, and
  // many on average (the counts fall fast once clusters merge): the next
  // pass skips the tiled scorer and scores every vertex by the wave
  ctl->defer_all = (2 * c[4] > c[2] && c[0] > 12 * c[2]) ? 1 : 0;
  ctl->passes += 1;
  ctl->evals += ctl->pass_evals;
  ctl->pass_evals = 0;
  ctl->dS2 = 0;
  ctl->dN2 = 0;
  if (ctl->nprop == 0) {
    ctl->converged = 1;
    ctl->done = 1;
    if (ctl->trace) {
      int64_t* r = ctl->trace + (int64_t)(ctl->passes - 1) * 4;
      r[0] = 0; r[1] = 0; r[2] = 0; r[3] = ctl->O;
    }
  }
}

// Apply the move of v (from -> to) with sign d (+1 apply, -1 undo) to the
// sizes and counts; lanes of the wave take the partitions.  Returns this
// lane's share of the change of the sums of squares (N part; the size part
// is added by lane 0 to *ds2).
__device__ inline int64_t move_counts(const PassArgs& a, int64_t v, int32_t from, int32_t to,
                                      int32_t d, int lane, int64_t* ds2) {
  int64_t acc = 0;
  const int32_t* row = a.Lvm + v * a.k;
  int32_t claimed = 0;  // these keys exist already (k_apply_all added them)
  for (int i = lane; i < a.k; i += 64) {
    const int32_t l = row[i];
    int32_t o1 = atomicAdd(counter(a.t, cell_upd(a.t, i, to, l, claimed)), d);
    int32_t o2 = atomicAdd(counter(a.t, cell_upd(a.t, i, from, l, claimed)), -d);
    acc += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
  }
  if (claimed) atomicAdd(a.t.hocc, claimed);
  if (lane == 0) {
    int32_t o1 = atomicAdd(&a.s[to], d);
    int32_t o2 = atomicAdd(&a.s[from], -d);
    *ds2 += 2 * (int64_t)o1 * d + 1 - 2 * (int64_t)o2 * d + 1;
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Apply every proposal with per-workgroup aggregation.  Updates are keyed by
// table cell (sizes use keys cells + cluster) and summed in an LDS hash
// before one global atomic per distinct key.  Once half the slots hold keys
// the table takes no new ones (probe runs stay short when a workgroup sees
// many distinct keys, as on a first pass): a key not in it, or that finds no
// free slot within kHashProbe steps, goes straight to the global counter.
// A net update d on a counter whose previous value is `old` changes its
// square by 2 old d + d^2, so the flush measures the objective change
// exactly, whichever updates of a key went where.
// ---------------------------------------------------------------------------
constexpr int kHashSlots = 4096;
constexpr int kHashOpen = kHashSlots / 2;  // keys the table takes
constexpr int kHashProbe = 32;

// The changes of the sums of squares caused by one global update: the
// contingency part (n) and the size part (s).  Returned by value: pointers
// to the caller's accumulators would keep them in scratch memory.
struct Sq2 {
  int64_t n, s;
};

// Keys: [0, cells) table cells, [cells, cells + K0) cluster sizes,
// [cells + K0, cells + 2 K0) per-cluster move counts (churn_w).
__device__ __attribute__((always_inline)) inline Sq2 agg_add(int32_t* hkey, int32_t* hval,
                                                           int32_t* fill, const PassArgs& a,
                                                           int32_t* churn_w, int64_t key,
                                                           int32_t d) {
  const int32_t k32 = (int32_t)key;
  uint32_t h = ((uint32_t)k32 * 2654435761u) >> 20;  // 12 bits: kHashSlots
#pragma unroll 1
  for (int q = 0; q < kHashProbe; ++q) {
    int32_t cur = hkey[h];
    if (cur == -1) {
      if (*fill >= kHashOpen) break;  // the key is not in the table
      cur = atomicCAS(&hkey[h], -1, k32);
      if (cur == -1) {
        atomicAdd(fill, 1);
        cur = k32;
      }
    }
    if (cur == k32) {
      atomicAdd(&hval[h], d);
      return Sq2{0, 0};
    }
    h = (h + 1) & (kHashSlots - 1);
  }
  if (key < a.cells) {
    const int32_t old = atomicAdd(counter(a.t, (uint32_t)key), d);
    return Sq2{2 * (int64_t)old * d + 1, 0};
  }
  if (key < a.cells + a.K0) {
    const int32_t old = atomicAdd(&a.s[key - a.cells], d);
    return Sq2{0, 2 * (int64_t)old * d + 1};
  }
  atomicAdd(&churn_w[key - a.cells - a.K0], d);
  return Sq2{0, 0};
}

// The proposers of the pass, in plist (order irrelevant): one atomic per
// chunk of V kBlock vertices.
__global__ __launch_bounds__(kBlock) void k_props(PassArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  __shared__ int32_t s_base;
  constexpr int V = 4;
  constexpr int64_t kChunk = (int64_t)V * kBlock;
  const int t = threadIdx.x;
  int64_t rows = 0;  // hashed rows: the rows the proposals can add
  for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < a.n; c0 += (int64_t)gridDim.x * kChunk) {
    bool pr[V];
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t v = c0 + j * kBlock + t;
      pr[j] = v < a.n && a.prop[v] >= 0;
      mine += pr[j];
      if (pr[j] && a.rdist) rows += a.rdist[v];
    }
    int32_t total;
    int32_t off = block_exclusive_scan(mine, &total);
    if (t == 0 && total) s_base = atomicAdd(&ctl->plist_count, total);
    __syncthreads();
    if (total) {
      off += s_base;
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (pr[j]) a.plist[off++] = (int32_t)(c0 + j * kBlock + t);
    }
    __syncthreads();
  }
  if (a.rdist) {  // one atomic per workgroup
    __shared__ int64_t s_rows[kBlock / 64];
    rows = wave_sum64(rows);
    if ((t & 63) == 0) s_rows[t >> 6] = rows;
    __syncthreads();
    if (t == 0) {
      int64_t tot = 0;
      for (int j = 0; j < kBlock / 64; ++j) tot += s_rows[j];
      if (tot) atomicAdd((unsigned long long*)&ctl->prop_rows, (unsigned long long)tot);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_apply_all(PassArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  const int64_t count = ctl->plist_count;
  const int64_t active = gridDim.x;
  __shared__ int32_t hkey[kHashSlots];
  __shared__ int32_t hval[kHashSlots];
  __shared__ int32_t fill;
  for (int j = threadIdx.x; j < kHashSlots; j += kBlock) {
    hkey[j] = -1;
    hval[j] = 0;
  }
  if (threadIdx.x == 0) fill = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  int64_t dn2 = 0, ds2 = 0;
  int32_t claimed = 0;
  // moves per cluster, read by the next pass's scorer (counted over every
  // proposal: a fallback pass commits fewer, so the count is an upper bound)
  int32_t* churn_w = a.churn ? a.churn + (int64_t)(ctl->passes & 1) * a.K0 : nullptr;
  // the wave serves the proposals of its 64 vertices four at a time, one
  // per group of 16 lanes, the lanes of a group spread over the partitions
  constexpr int kApplyLanes = 16;
  const int grp = lane / kApplyLanes, gl = lane % kApplyLanes;
  // the listed proposers, 64 at a time per wave of the active workgroups
  const int64_t nact = active * (kBlock / 64);
  for (int64_t e0 = wave * 64; e0 < count; e0 += nact * 64) {
    const int64_t e = e0 + lane;
    const int32_t vl = e < count ? a.plist[e] : 0;
    const int32_t p = e < count ? a.prop[vl] : kNone;
    uint64_t mask = __ballot(p >= 0);
    while (mask) {
      uint64_t m = mask;  // this group's proposal: the grp-th selected entry
      for (int q = 0; q < grp; ++q) m &= m - 1;
      const int b = m ? __ffsll((unsigned long long)m) - 1 : -1;
      for (int q = 0; q < 64 / kApplyLanes; ++q) mask &= mask - 1;
      const int32_t to = __shfl(p, b < 0 ? 0 : b, 64);
      const int64_t w = __shfl(vl, b < 0 ? 0 : b, 64);
      if (b < 0) continue;
      const int32_t from = a.C[w];
      const int32_t* row = a.Lvm + w * a.k;
      for (int i = gl; i < a.k; i += kApplyLanes) {
        const int32_t l = row[i];
        const Sq2 up =
            agg_add(hkey, hval, &fill, a, churn_w, cell_upd(a.t, i, to, l, claimed), +1);
        const Sq2 dn =
            agg_add(hkey, hval, &fill, a, churn_w, cell_upd(a.t, i, from, l, claimed), -1);
        dn2 += up.n + dn.n;
      }
      if (gl == 0) {
        const Sq2 up = agg_add(hkey, hval, &fill, a, churn_w, a.cells + to, +1);
        const Sq2 dn = agg_add(hkey, hval, &fill, a, churn_w, a.cells + from, -1);
        ds2 += up.s + dn.s;
      } else if (gl == 1 && churn_w) {
        agg_add(hkey, hval, &fill, a, churn_w, a.cells + a.K0 + to, +1);
        agg_add(hkey, hval, &fill, a, churn_w, a.cells + a.K0 + from, +1);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kHashSlots; j += kBlock) {
    const int32_t key = hkey[j], d = hval[j];
    if (key < 0 || d == 0) continue;
    if (key < a.cells) {
      const int32_t old = atomicAdd(counter(a.t, (uint32_t)key), d);
      dn2 += 2 * (int64_t)old * d + (int64_t)d * d;
    } else if (key < a.cells + a.K0) {
      const int32_t old = atomicAdd(&a.s[key - a.cells], d);
      ds2 += 2 * (int64_t)old * d + (int64_t)d * d;
    } else {
      atomicAdd(&churn_w[key - a.cells - a.K0], d);
    }
  }
  if (a.t.hashed) flush_claims(a.t, claimed);
  dn2 = wave_sum64(dn2);
  ds2 = wave_sum64(ds2);
  if (lane == 0) {
    if (dn2) atomicAdd((unsigned long long*)&ctl->dN2, (unsigned long long)dn2);
    if (ds2) atomicAdd((unsigned long long*)&ctl->dS2, (unsigned long long)ds2);
  }
}

// ---------------------------------------------------------------------------
// Batch apply for dense tables whose per-partition slice fits in LDS.  The
// grid is (slices, k): workgroup (p, i) takes slice p of the listed
// proposals and histograms partition i's count changes in LDS, +1 at
// (to, l) and -1 at (from, l) with l the mover's label in partition i; then
// it adds every nonzero change to the table with one atomic, whose returned
// value gives the cell's exact share of the change of the sum of squares
// (2 old d + d^2 for each addition, which sums to the exact change whatever
// the order).  The workgroups of partition 0 do the same for the cluster
// sizes and count the moves per cluster (churn).  Late passes, whose few
// proposals mostly move between the same clusters, run one slice: each
// counter then receives one atomic.
// ---------------------------------------------------------------------------
constexpr int kDeltaPerSlice = 2048;  // proposals per slice of the list
constexpr int kDeltaUnroll = 4;

template <bool IL>
__global__ __launch_bounds__(kBlock) void k_apply_delta(PassArgs a) {
  extern __shared__ int32_t sh[];
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  const int64_t count = ctl->plist_count;
  const int64_t active = min((int64_t)gridDim.x,
                             max((int64_t)1, (count + kDeltaPerSlice - 1) / kDeltaPerSlice));
  const int p = blockIdx.x, i = blockIdx.y, t = threadIdx.x;
  if (p >= active || count == 0) return;
  const int32_t k = a.k, K0 = a.K0;
  const int32_t Li = IL ? a.t.Lmax : a.t.L[i];
  const int32_t cells = K0 * Li;  // fits in LDS (checked by the host)
  const bool sizes = i == 0;
  int32_t* hd = sh;
  int32_t* hs = sh + cells;
  int32_t* hc = hs + K0;
  const int32_t zero_len = sizes ? cells + 2 * K0 : cells;
  for (int32_t j = t; j < zero_len; j += kBlock) sh[j] = 0;
  __syncthreads();
  const int64_t per = (count + active - 1) / active;
  const int64_t eb = (int64_t)p * per, ee = min(count, eb + per);
  for (int64_t e0 = eb + t; e0 < ee; e0 += (int64_t)kDeltaUnroll * kBlock) {
    int32_t vv[kDeltaUnroll], to[kDeltaUnroll], fr[kDeltaUnroll], lb[kDeltaUnroll];
#pragma unroll
    for (int q = 0; q < kDeltaUnroll; ++q) {
      const int64_t e = e0 + (int64_t)q * kBlock;
      vv[q] = e < ee ? a.plist[e] : -1;
    }
#pragma unroll
    for (int q = 0; q < kDeltaUnroll; ++q) {
      if (vv[q] < 0) continue;
      to[q] = a.prop[vv[q]];
      fr[q] = a.C[vv[q]];
      lb[q] = a.Lvm[(int64_t)vv[q] * k + i];
    }
#pragma unroll
    for (int q = 0; q < kDeltaUnroll; ++q) {
      if (vv[q] < 0) continue;
      atomicAdd(&hd[to[q] * Li + lb[q]], 1);
      atomicAdd(&hd[fr[q] * Li + lb[q]], -1);
      if (sizes) {
        atomicAdd(&hs[to[q]], 1);
        atomicAdd(&hs[fr[q]], -1);
        atomicAdd(&hc[to[q]], 1);
        atomicAdd(&hc[fr[q]], 1);
      }
    }
  }
  __syncthreads();
  int64_t dn2 = 0, ds2 = 0;
  const int64_t toff = IL ? 0 : a.t.toff[i];
  for (int32_t j0 = t; j0 < cells; j0 += kDeltaUnroll * kBlock) {
    int32_t d[kDeltaUnroll], old[kDeltaUnroll];
#pragma unroll
    for (int q = 0; q < kDeltaUnroll; ++q) {
      const int32_t j = j0 + q * kBlock;
      d[q] = j < cells ? hd[j] : 0;
      old[q] = 0;
      if (d[q]) {
        const int32_t x = j / Li, l = j - x * Li;
        const uint32_t c = IL ? ((uint32_t)x * (uint32_t)Li + (uint32_t)l) * (uint32_t)k + i
                              : (uint32_t)toff + (uint32_t)j;
        old[q] = atomicAdd(&a.t.N[c], d[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kDeltaUnroll; ++q)
      dn2 += 2 * (int64_t)old[q] * d[q] + (int64_t)d[q] * d[q];
  }
  if (sizes) {
    int32_t* churn_w = a.churn ? a.churn + (int64_t)(ctl->passes & 1) * K0 : nullptr;
    for (int32_t x = t; x < K0; x += kBlock) {
      const int32_t d = hs[x];
      if (d) {
        const int32_t old = atomicAdd(&a.s[x], d);
        ds2 += 2 * (int64_t)old * d + (int64_t)d * d;
      }
      if (churn_w && hc[x]) atomicAdd(&churn_w[x], hc[x]);
    }
  }
  dn2 = wave_sum64(dn2);
  ds2 = wave_sum64(ds2);
  __shared__ int64_t red[2][kBlock / 64];
  if ((t & 63) == 0) {
    red[0][t >> 6] = dn2;
    red[1][t >> 6] = ds2;
  }
  __syncthreads();
  if (t == 0) {
    int64_t n2 = 0, s2 = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      n2 += red[0][w];
      s2 += red[1][w];
    }
    if (n2) atomicAdd((unsigned long long*)&ctl->dN2, (unsigned long long)n2);
    if (s2) atomicAdd((unsigned long long*)&ctl->dS2, (unsigned long long)s2);
  }
}

// Vertex w moved: it and its out-neighbours (its in-neighbours, the graph
// being symmetric) recompute their candidate sets next pass.
__device__ inline void mark_dirty(const PassArgs& a, int64_t w, int lane) {
  if (!a.dirty) return;
  if (lane == 0) a.dirty[w] = 1;
  const int64_t b = a.row_ptr[w], e = a.row_ptr[w + 1];
  for (int64_t p = b + lane; p < e; p += 64) a.dirty[a.col[p]] = 1;
}

// Vertex w now sits in cluster c: every arc pointing at w learns it.
__device__ inline void relabel_in_arcs(const PassArgs& a, int64_t w, int32_t c, int lane) {
  if (!a.ac) return;
  const int32_t b = a.in_ptr[w], e = a.in_ptr[w + 1];
  for (int32_t p = b + lane; p < e; p += 64) a.ac[a.in_pos[p]] = c;
}

// The apply-type kernels walk the vertices 64 at a time per wave: one
// coalesced load of the proposals, a ballot, then the wave serves each
// selected vertex with its lanes spread over the partitions.
enum ApplyMode { kApplyAll = 0, kCommitOrElect = 1, kFallbackCommit = 2, kFallbackFinish = 3 };

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_apply(PassArgs a) {
  Ctl* ctl = a.ctl;
  if (ctl->done) return;
  if ((MODE == kFallbackCommit || MODE == kFallbackFinish) && !ctl->fallback) return;
  const bool fb = ctl->fallback;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) / 64;
  int64_t dn2 = 0, ds2 = 0;
  int32_t committed = 0;
  for (int64_t v0 = wave * 64; v0 < a.n; v0 += nwaves * 64) {
    const int64_t v = v0 + lane;
    int32_t p = v < a.n ? a.prop[v] : kNone;
    bool sel;
    if (MODE == kFallbackFinish) sel = p != kNone;  // committed (>= 0) or not (<= -2)
    else sel = p >= 0;
    uint64_t mask = __ballot(sel);
    while (mask) {
      const int b = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const int64_t w = v0 + b;
      const int32_t pw = __shfl(p, b, 64);
      const int32_t from = a.C[w];
      if (MODE == kApplyAll) {
        dn2 += move_counts(a, w, from, pw, +1, lane, &ds2);
      } else if (MODE == kCommitOrElect) {
        if (!fb) {
          if (lane == 0) {
            a.C[w] = pw;
            cn_store(a, w, pw);
          }
          relabel_in_arcs(a, w, pw, lane);
          mark_dirty(a, w, lane);
        } else {
          move_counts(a, w, from, pw, -1, lane, &ds2);  // undo the batch
          if (lane == 0) {
            const uint64_t key = owner_key(a.dprop[w], w);
            atomicMin((unsigned long long*)&a.owner[from], (unsigned long long)key);
            atomicMin((unsigned long long*)&a.owner[pw], (unsigned long long)key);
          }
        }
      } else if (MODE == kFallbackCommit) {
        const uint64_t key = owner_key(a.dprop[w], w);
        const bool own = a.owner[from] == key && a.owner[pw] == key;
        if (own) {
          dn2 += move_counts(a, w, from, pw, +1, lane, &ds2);
          if (lane == 0) ++committed;
        } else if (lane == 0) {
          a.prop[w] = -2 - pw;  // proposal kept out of this pass
        }
      } else {  // kFallbackFinish
        const int32_t to = pw >= 0 ? pw : -2 - pw;
        if (lane == 0) {
          a.owner[from] = ~0ull;
          a.owner[to] = ~0ull;
          if (pw >= 0) {
            a.C[w] = pw;
            cn_store(a, w, pw);
          }
        }
        if (pw >= 0) {
          relabel_in_arcs(a, w, pw, lane);
          mark_dirty(a, w, lane);
        }
      }
    }
  }
  if (MODE == kApplyAll || MODE == kFallbackCommit) {
    dn2 = wave_sum64(dn2);
    ds2 = wave_sum64(ds2);
    committed = wave_sum32(committed);
    if (lane == 0) {
      if (dn2) atomicAdd((unsigned long long*)&ctl->dN2, (unsigned long long)dn2);
      if (ds2) atomicAdd((unsigned long long*)&ctl->dS2, (unsigned long long)ds2);
      if (committed) atomicAdd(&ctl->committed, committed);
    }
  }
}

// Hashed tables: before the batch is applied, rebuild the table from the
// partition (the counts are a function of C alone) if the keys the batch may
// add could take it beyond half full.  Keys: the batch adds at most k keys
// per proposal; the table holds 4 n k slots or more and at most n k live
// keys, so after a rebuild there is always room.  Rows: a proposal adds at
// most its vertex's distinct label ids, at most T0 in all, over at most T0
// live rows, in more than 2 T0 rows.  The first pass's table is the one
// just built (no key without a count), so a rebuild would not change it.
__global__ void k_hash_guard(PassArgs a, int64_t limit) {
  Ctl* ctl = a.ctl;
  if (ctl->done) {
    *a.hflag = 0;
    return;
  }
  // keys the batch may add: k a proposal, or for hashed rows the distinct
  // label ids of the proposers (the rows a move can add)
  const int64_t adds = a.t.rows ? ctl->prop_rows : (int64_t)a.k * ctl->nprop;
  const bool need = ctl->passes > 1 && (int64_t)*a.t.hocc + adds > limit;
  *a.hflag = need ? 1 : 0;
  if (need) *a.t.hocc = 0;
}

__global__ __launch_bounds__(kBlock) void k_hash_reset(PassArgs a) {
  if (!*a.hflag) return;
  if (a.t.rows) {  // empty keys, zero counts
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j <= (int64_t)a.t.hmask;
         j += (int64_t)gridDim.x * kBlock)
      a.t.rkeys[j] = kHashEmpty;
    const int64_t cells = ((int64_t)a.t.hmask + 1) * a.k;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < cells;
         j += (int64_t)gridDim.x * kBlock)
      a.t.N[j] = 0;
    return;
  }
  uint4* H = reinterpret_cast<uint4*>(a.t.N);
  const uint4 empty = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j <= (int64_t)a.t.hmask;
       j += (int64_t)gridDim.x * kBlock)
    H[j] = empty;
}

__global__ __launch_bounds__(kBlock) void k_hash_refill(PassArgs a) {
  if (!*a.hflag) return;
  if (a.t.rows) {
    flush_claims(a.t, rows_count(a.t, a.C, a.Lvm, a.n, a.k,
                                 (int64_t)blockIdx.x * kBlock + threadIdx.x,
                                 (int64_t)gridDim.x * kBlock));
    return;
  }
  const int64_t total = a.n * a.k;
  int32_t claimed = 0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total;
       j += (int64_t)gridDim.x * kBlock) {
    const int64_t v = j / a.k;
    const int i = (int)(j - v * a.k);
    atomicAdd(counter(a.t, cell_upd(a.t, i, a.C[v], a.Lvm[j], claimed)), 1);
  }
  flush_claims(a.t, claimed);
}

// Member lists of the clusters at the start of the pass (mstart holds the
// exclusive scan of the sizes, mcnt is zeroed): a counting sort of C.
__global__ __launch_bounds__(kBlock) void k_member_fill(PassArgs a) {
  if (a.ctl->done) return;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < a.n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t x = a.C[v];
    if (a.s[x] <= a.msum_max)  // larger clusters are probed, not listed
      a.members[a.mstart[x] + atomicAdd(&a.mcnt[x], 1)] = (int32_t)v;
  }
}

__global__ void k_decide(Ctl* ctl) {
  if (ctl->done) return;
  const int64_t dO = (int64_t)ctl->k * ctl->dS2 - 2 * ctl->dN2;
  ctl->dS2 = 0;
  ctl->dN2 = 0;
  if (dO < 0) {
    ctl->fallback = 0;
    ctl->O += dO;
    ctl->committed = ctl->nprop;
  } else {
    ctl->fallback = 1;
    ctl->fallback_rounds += 1;
    ctl->committed = 0;
  }
}

__global__ void k_end(Ctl* ctl) {
  if (ctl->done) return;
  if (ctl->fallback) ctl->O += (int64_t)ctl->k * ctl->dS2 - 2 * ctl->dN2;
  ctl->moves += ctl->committed;
  if (ctl->trace) {
    int64_t* r = ctl->trace + (int64_t)(ctl->passes - 1) * 4;
    r[0] = ctl->nprop;
    r[1] = ctl->committed;
    r[2] = ctl->fallback;
    r[3] = ctl->O;
  }
  ctl->nprop = 0;
  ctl->committed = 0;
  ctl->fallback = 0;
  ctl->heavy_count = 0;
  ctl->rescore_count = 0;
  ctl->plist_count = 0;
  ctl->prop_rows = 0;
  ctl->dS2 = 0;
  ctl->dN2 = 0;
  if (ctl->passes >= ctl->max_rounds) ctl->done = 1;
}

__global__ void k_ctl_init(Ctl* ctl, const int64_t* acc, int32_t k, int32_t max_rounds,
                           int64_t* trace) {
  Ctl c = {};
  c.k = k;
  c.max_rounds = max_rounds;
  c.trace = trace;
  c.O = (int64_t)k * acc[0] + acc[1] - 2 * acc[2];
  *ctl = c;
}

template <int G>
void launch_score(const PassArgs& a, int grid, hipStream_t st) {
  k_score<G, false><<<grid, kBlock, 0, st>>>(a);
}

template <int TK>
void launch_tile(const PassArgs& a, int grid, hipStream_t st) {
  if (a.ac) k_score_tile<0, TK><<<grid, kBlock, 0, st>>>(a);
  else if (a.cn_bytes == 1) k_score_tile<1, TK><<<grid, kBlock, 0, st>>>(a);
  else if (a.cn_bytes == 2) k_score_tile<2, TK><<<grid, kBlock, 0, st>>>(a);
  else k_score_tile<4, TK><<<grid, kBlock, 0, st>>>(a);
  if (!a.st) return;
  if (a.ac) k_score_list<0, TK><<<grid, kBlock, 0, st>>>(a);
  else if (a.cn_bytes == 1) k_score_list<1, TK><<<grid, kBlock, 0, st>>>(a);
  else if (a.cn_bytes == 2) k_score_list<2, TK><<<grid, kBlock, 0, st>>>(a);
  else k_score_list<4, TK><<<grid, kBlock, 0, st>>>(a);
}

}  // namespace

bool score_lanes_ok(int lanes) {
  return lanes == 0 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 || lanes == 64;
}

void launch_ctl_init(Ctl* ctl, const int64_t* acc, int32_t k, int32_t max_rounds,
                     int64_t* trace, hipStream_t st) {
  k_ctl_init<<<1, 1, 0, st>>>(ctl, acc, k, max_rounds, trace);
}

void enqueue_pass(const PassArgs& a, int lanes, int grid_score, int grid_apply, hipStream_t st,
                  hipEvent_t score_begin, hipEvent_t score_end) {
  if (a.members) {
    launch_scan(a.s, a.mstart, a.K0, a.mscan_tmp, st);
    launch_fill_i32(a.mcnt, a.K0, 0, st);
    k_member_fill<<<grid_apply, kBlock, 0, st>>>(a);
  }
  if (score_begin) (void)hipEventRecord(score_begin, st);
  switch (lanes) {
    case 0:
      if (a.st) k_status<<<grid_apply, kBlock, 0, st>>>(a);
      if (a.t.hashed) launch_tile<kHashed>(a, grid_score, st);
      else if (a.t.interleaved) launch_tile<kInterleaved>(a, grid_score, st);
      else launch_tile<kBlocked>(a, grid_score, st);
      // deferred vertices: one per wave, as many waves as the chip holds
      k_score<64, true><<<grid_score, kBlock, 0, st>>>(a);
      break;
    case 4: launch_score<4>(a, grid_score, st); break;
    case 8: launch_score<8>(a, grid_score, st); break;
    case 16: launch_score<16>(a, grid_score, st); break;
    case 32: launch_score<32>(a, grid_score, st); break;
    default: launch_score<64>(a, grid_score, st); break;
  }
  if (score_end) (void)hipEventRecord(score_end, st);
  k_begin<<<1, 1, 0, st>>>(a.ctl, a.pc);
  k_props<<<grid_apply, kBlock, 0, st>>>(a);
  if (a.t.hashed) {
    k_hash_guard<<<1, 1, 0, st>>>(a, (int64_t)((a.t.hmask + 1) / 2));
    k_hash_reset<<<grid_apply, kBlock, 0, st>>>(a);
    k_hash_refill<<<grid_apply, kBlock, 0, st>>>(a);
  }
  if (a.delta_lds > 0) {
    const dim3 grid((unsigned)a.delta_slices, (unsigned)a.k);
    if (a.t.interleaved) k_apply_delta<true><<<grid, kBlock, a.delta_lds, st>>>(a);
    else k_apply_delta<false><<<grid, kBlock, a.delta_lds, st>>>(a);
  } else {
    k_apply_all<<<grid_apply, kBlock, 0, st>>>(a);
  }
  k_decide<<<1, 1, 0, st>>>(a.ctl);
  k_apply<kCommitOrElect><<<grid_apply, kBlock, 0, st>>>(a);
  k_apply<kFallbackCommit><<<grid_apply, kBlock, 0, st>>>(a);
  k_apply<kFallbackFinish><<<grid_apply, kBlock, 0, st>>>(a);
  k_end<<<1, 1, 0, st>>>(a.ctl);
}

}  // namespace mcc
