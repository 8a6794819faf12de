// Partition comparison on the device (Results, "Evaluation metrics";
// Methods, "Grouping homogeneous partitions"): from the contingency counts
// n_ab of two partitions A and B,
//   split-join distance  2n - sum_a max_b n_ab - sum_b max_a n_ab,
//   variation of information
//       (sum_a n_a ln n_a + sum_b n_b ln n_b - 2 sum_ab n_ab ln n_ab) / n,
//   Rand distance        Mirkin(A, B) / (n (n - 1)),
// and the split-join distance of every pair of k partitions at once.
#include "impl.h"

namespace mcc {

namespace {

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

template <typename T>
__device__ T block_total(T x, T* part /* kBlock / 64 */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  T t = 0;
#pragma unroll
  for (int j = 0; j < kBlock / 64; ++j) t += part[j];  // fixed order: same bits every run
  __syncthreads();
  return t;
}

__device__ inline double xlogx(int32_t c) { return c > 0 ? (double)c * log((double)c) : 0.0; }

// One pass over the cells of a k = 1 table (A = clusters, B = labels):
// row and column maxima, column sums, and per-block sums of c ln c.
__global__ __launch_bounds__(kBlock) void k_cell_stats(Tables t, int64_t cells, int32_t Lb,
                                                       int32_t* __restrict__ rowmax,
                                                       int32_t* __restrict__ colmax,
                                                       int32_t* __restrict__ colsum,
                                                       double* __restrict__ partial) {
  __shared__ double part[kBlock / 64];
  double acc = 0.0;
  const uint32_t g0 = t.hashed ? (uint32_t)t.toff[0] : 0u;
  for (int64_t j = gtid(); j < cells; j += gstride()) {
    int32_t x, l, c;
    if (t.hashed) {
      const uint4 e = reinterpret_cast<const uint4*>(t.N)[j];
      if (e.x == 0xffffffffu && e.y == 0xffffffffu) continue;
      c = (int32_t)e.z;
      x = (int32_t)e.y;
      l = (int32_t)(e.x - g0);
    } else {
      c = t.N[j];
      x = (int32_t)(j / Lb);
      l = (int32_t)(j - (int64_t)x * Lb);
    }
    if (c == 0) continue;
    atomicMax(rowmax + x, c);
    atomicMax(colmax + l, c);
    atomicAdd(colsum + l, c);
    acc += xlogx(c);
  }
  acc = block_total(acc, part);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_xlogx(const int32_t* __restrict__ a, int64_t len,
                                                  double* __restrict__ partial) {
  __shared__ double part[kBlock / 64];
  double acc = 0.0;
  for (int64_t j = gtid(); j < len; j += gstride()) acc += xlogx(a[j]);
  acc = block_total(acc, part);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// out[0] = sum of partial[0 .. count) in a fixed order
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partial,
                                                         int32_t count, double* __restrict__ out) {
  __shared__ double part[kBlock / 64];
  double acc = 0.0;
  for (int32_t j = threadIdx.x; j < count; j += kBlock) acc += partial[j];
  acc = block_total(acc, part);
  if (threadIdx.x == 0) out[0] = acc;
}

__global__ __launch_bounds__(kBlock) void k_sum_i32(const int32_t* __restrict__ a, int64_t len,
                                                    int64_t* __restrict__ acc) {
  __shared__ int64_t part[kBlock / 64];
  int64_t s = 0;
  for (int64_t j = gtid(); j < len; j += gstride()) s += a[j];
  s = block_total(s, part);
  if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)acc, (unsigned long long)s);
}

// Pair tables: T[poff[p] + a * L[j] + b] = #{v : D_i(v) = a, D_j(v) = b}
// for the pair p = (pi[p], pj[p]); D is partition-major dense label ids.
// A pair whose table fits kPairLds entries is counted in LDS first.
constexpr int kPairLds = 16384;

__global__ __launch_bounds__(kBlock) void k_pair_hist(const int32_t* __restrict__ D, int64_t n,
                                                      const int32_t* __restrict__ pi,
                                                      const int32_t* __restrict__ pj,
                                                      const int64_t* __restrict__ poff,
                                                      const int32_t* __restrict__ L,
                                                      int32_t npairs, int32_t* __restrict__ T) {
  __shared__ int32_t h[kPairLds];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per;
  const int64_t v1 = min(n, v0 + per);
  for (int32_t p = blockIdx.y; p < npairs; p += gridDim.y) {
    const int32_t i = pi[p], j = pj[p];
    const int32_t Lj = L[j];
    const int64_t cells = (int64_t)L[i] * Lj;
    const bool lds = cells <= kPairLds;
    int32_t* Tp = T + poff[p];
    if (lds) {
      for (int64_t c = threadIdx.x; c < cells; c += kBlock) h[c] = 0;
      __syncthreads();
    }
    const int32_t* Di = D + (int64_t)i * n;
    const int32_t* Dj = D + (int64_t)j * n;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += kBlock) {
      const int64_t c = (int64_t)Di[v] * Lj + Dj[v];
      if (lds) atomicAdd(&h[c], 1);
      else atomicAdd(&Tp[c], 1);
    }
    if (lds) {
      __syncthreads();
      for (int64_t c = threadIdx.x; c < cells; c += kBlock)
        if (h[c]) atomicAdd(&Tp[c], h[c]);
      __syncthreads();
    }
  }
}

// dist[p] = split-join distance of pair p from its table
__global__ __launch_bounds__(kBlock) void k_pair_split_join(const int32_t* __restrict__ T,
                                                            const int32_t* __restrict__ pi,
                                                            const int32_t* __restrict__ pj,
                                                            const int64_t* __restrict__ poff,
                                                            const int32_t* __restrict__ L,
                                                            int32_t npairs, int64_t n,
                                                            int64_t* __restrict__ dist) {
  __shared__ int64_t part[kBlock / 64];
  for (int32_t p = blockIdx.x; p < npairs; p += gridDim.x) {
    const int32_t Li = L[pi[p]], Lj = L[pj[p]];
    const int32_t* Tp = T + poff[p];
    int64_t s = 0;
    for (int32_t a = threadIdx.x; a < Li; a += kBlock) {  // best label of j for each label of i
      int32_t m = 0;
      for (int32_t b = 0; b < Lj; ++b) m = max(m, Tp[(int64_t)a * Lj + b]);
      s += m;
    }
    for (int32_t b = threadIdx.x; b < Lj; b += kBlock) {  // and the other way round
      int32_t m = 0;
      for (int32_t a = 0; a < Li; ++a) m = max(m, Tp[(int64_t)a * Lj + b]);
      s += m;
    }
    s = block_total(s, part);
    if (threadIdx.x == 0) dist[p] = 2 * n - s;
  }
}

inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int cell_stats_blocks(int64_t cells) { return grid_for(cells, kBlock * 4, 2048); }
int xlogx_blocks(int64_t len) { return grid_for(len, kBlock * 4, 2048); }

void launch_cell_stats(const Tables& t, int64_t cells, int32_t Lb, int32_t* rowmax,
                       int32_t* colmax, int32_t* colsum, double* partial, hipStream_t st) {
  k_cell_stats<<<cell_stats_blocks(cells), kBlock, 0, st>>>(t, cells, Lb, rowmax, colmax, colsum,
                                                            partial);
}

void launch_xlogx(const int32_t* a, int64_t len, double* partial, hipStream_t st) {
  k_xlogx<<<xlogx_blocks(len), kBlock, 0, st>>>(a, len, partial);
}

void launch_sum_partials(const double* partial, int32_t count, double* out, hipStream_t st) {
  k_sum_partials<<<1, kBlock, 0, st>>>(partial, count, out);
}

void launch_sum_i32(const int32_t* a, int64_t len, int64_t* acc, hipStream_t st) {
  if (len > 0) k_sum_i32<<<grid_for(len, kBlock * 4, 1024), kBlock, 0, st>>>(a, len, acc);
}

void launch_pair_tables(const int32_t* D, int64_t n, const int32_t* pi, const int32_t* pj,
                        const int64_t* poff, const int32_t* L, int32_t npairs, int32_t* T,
                        hipStream_t st) {
  // a few workgroups per pair along the vertices, many pairs side by side
  const int chunks = grid_for(n, 16384, 64);
  dim3 g(chunks, (unsigned)std::min<int32_t>(npairs, 65535));
  k_pair_hist<<<g, kBlock, 0, st>>>(D, n, pi, pj, poff, L, npairs, T);
}

void launch_pair_split_join(const int32_t* T, const int32_t* pi, const int32_t* pj,
                            const int64_t* poff, const int32_t* L, int32_t npairs, int64_t n,
                            int64_t* dist, hipStream_t st) {
  k_pair_split_join<<<std::min<int32_t>(npairs, 65535), kBlock, 0, st>>>(T, pi, pj, poff, L,
                                                                         npairs, n, dist);
}

}  // namespace mcc
