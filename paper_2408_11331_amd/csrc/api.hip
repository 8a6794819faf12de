// Host side of libmcc: argument checks, the workspace cache, the setup
// sequence and the device-driven pass loop behind the C interface in
// include/mcc.h.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "impl.h"
#include "mcc.h"

namespace mcc {
// setup.hip
void launch_dense_map(const int32_t* in, int64_t n, const int32_t* scan, int32_t* out,
                      hipStream_t st);
// Hashed rows from clusters of one vertex each: the counts stored, not added.
void launch_build_rows_single(const int32_t* C, const int32_t* Lvm, int64_t n, int32_t k,
                              Tables t, hipStream_t st);
}

namespace {

using namespace mcc;

thread_local std::string g_hip_error;

// Largest label flag array (sum over partitions of max label + 1) and
// largest dense table (sum over partitions of clusters x labels) accepted.
constexpr int64_t kMaxLabelFlags = (int64_t)1 << 30;
constexpr int64_t kMaxTableEntries = (int64_t)3 << 29;  // 6 GiB of int32 counts
// Largest hashed table (16-byte slots; cell ids stay below 2^31).
constexpr int64_t kMaxHashSlots = (int64_t)1 << 30;

struct HipError {
  hipError_t e;
};

inline void hipck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    g_hip_error = std::string(what) + ": " + hipGetErrorString(e);
    throw HipError{e};
  }
}
#define HIPCK(x) hipck((x), #x)

struct NoMem {};
struct Status {
  int code;
};

// Workspace chunks kept between calls, per device: an arena takes a cached
// chunk when it needs one and gives back what it took when it ends, so
// steady-state calls allocate and free nothing (allocation and free calls
// cost about a tenth of a millisecond each, large frees synchronise the
// device), and arenas nested in one call share the cache instead of each
// allocating anew.  An arena drains its stream before it returns its
// chunks, so a cached chunk is idle and any stream may take it: calls on
// several streams share one cache.  Chunks beyond kCachedMax bytes in total
// are freed on return; mcc_release_workspace frees the rest.
struct Chunk {
  void* p;
  size_t size;
};

struct ChunkCache {
  std::mutex m;
  std::map<int, std::vector<Chunk>> free;  // per device
  size_t bytes = 0;
};

ChunkCache& chunk_cache() {
  static ChunkCache* c = new ChunkCache;  // never destroyed: may outlive static teardown
  return *c;
}

constexpr size_t kCachedMax = (size_t)64 << 30;

// Frees the cached (idle) chunks of device `dev`, which is current.
void release_cached(int dev) {
  ChunkCache& c = chunk_cache();
  std::lock_guard<std::mutex> lock(c.m);
  for (auto it = c.free.begin(); it != c.free.end();) {
    if (it->first != dev) {
      ++it;
      continue;
    }
    for (const Chunk& k : it->second) {
      (void)hipFree(k.p);
      c.bytes -= k.size;
    }
    it = c.free.erase(it);
  }
}

class Arena {
 public:
  explicit Arena(hipStream_t st) : st_(st) { (void)hipGetDevice(&dev_); }
  // An arena over a fixed device region of `cap` bytes: get() carves from
  // it and throws Status{MCC_ESCRATCH} when it is full; nothing is
  // allocated, freed or cached.
  Arena(hipStream_t st, unsigned char* fixed, size_t cap)
      : st_(st), fixed_(fixed != nullptr), next_(fixed), left_(fixed ? cap : 0),
        fixed_cap_(fixed ? cap : 0) {
    (void)hipGetDevice(&dev_);
  }
  ~Arena() {
    // kernels and queued copies may still use the chunks: drain first
    (void)hipStreamSynchronize(st_);
    if (fixed_ || used_.empty()) return;
    ChunkCache& c = chunk_cache();
    std::lock_guard<std::mutex> lock(c.m);
    std::vector<Chunk>& keep = c.free[dev_];
    for (const Chunk& k : used_) {
      if (c.bytes + k.size <= kCachedMax) {
        keep.push_back(k);
        c.bytes += k.size;
      } else {
        (void)hipFree(k.p);
      }
    }
  }
  // Device bytes the arena holds: the chunks taken, or the fixed region's
  // carved part.
  size_t bytes_used() const {
    if (fixed_) return fixed_cap_ - left_;
    size_t b = 0;
    for (const Chunk& k : used_) b += k.size;
    return b;
  }
  // Host buffer that lives as long as the arena (source of async copies).
  template <class T>
  T* host(const std::vector<T>& src) {
    staging_.emplace_back(src.size() * sizeof(T) + 1);
    memcpy(staging_.back().data(), src.data(), src.size() * sizeof(T));
    return reinterpret_cast<T*>(staging_.back().data());
  }
  // Device buffer of `count` elements, 256-byte aligned.  Requests are
  // carved from chunks of kChunk bytes (a larger request gets a chunk of its
  // own), taken from the stream's cached chunks when one is large enough.
  template <class T>
  T* get(int64_t count) {
    if (count < 1) count = 1;
    const size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
    if (bytes <= left_) {
      void* r = next_;
      next_ += bytes;
      left_ -= bytes;
      return static_cast<T*>(r);
    }
    if (fixed_) throw Status{MCC_ESCRATCH};
    const Chunk k = chunk(std::max(bytes, kChunk));
    if (bytes >= kChunk) return static_cast<T*>(k.p);  // own chunk; keep the current one
    next_ = static_cast<unsigned char*>(k.p) + bytes;
    left_ = k.size - bytes;
    return static_cast<T*>(k.p);
  }

 private:
  // The smallest cached chunk of the device of at least `size` bytes, else
  // a new one.
  Chunk chunk(size_t size) {
    Chunk k{nullptr, 0};
    {
      ChunkCache& c = chunk_cache();
      std::lock_guard<std::mutex> lock(c.m);
      auto it = c.free.find(dev_);
      if (it != c.free.end()) {
        std::vector<Chunk>& v = it->second;
        size_t best = v.size();
        for (size_t j = 0; j < v.size(); ++j)
          if (v[j].size >= size && (best == v.size() || v[j].size < v[best].size)) best = j;
        if (best < v.size()) {
          k = v[best];
          v.erase(v.begin() + best);
          c.bytes -= k.size;
          if (v.empty()) c.free.erase(it);
        }
      }
    }
    if (!k.p) {
      void* p = nullptr;
      hipError_t e = hipMalloc(&p, size);
      if (e == hipErrorOutOfMemory) {
        // free every idle cached chunk of the device (any stream) and retry once
        (void)hipGetLastError();
        release_cached(dev_);
        e = hipMalloc(&p, size);
        if (e == hipErrorOutOfMemory) {
          (void)hipGetLastError();
          throw NoMem{};
        }
      }
      hipck(e, "hipMalloc");
      k = {p, size};
    }
    used_.push_back(k);
    return k;
  }

  static constexpr size_t kChunk = (size_t)16 << 20;
  hipStream_t st_;
  bool fixed_ = false;
  int dev_ = 0;
  std::vector<Chunk> used_;
  unsigned char* next_ = nullptr;
  size_t left_ = 0;
  size_t fixed_cap_ = 0;
  std::vector<std::vector<unsigned char>> staging_;
};

// Workspace of mcc_consensus_noalloc: one array per device, held from the
// library's first use on that device until the process ends.  Host code
// never passes the array's name to a kernel (on the host it names a
// stand-in, not device memory): it takes the device address once per device
// from hipGetSymbolAddress and uses that.
constexpr size_t kScratchBytes = (size_t)MCC_NOALLOC_SCRATCH_MIB << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_m;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
unsigned char* scratch_address() {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Status{MCC_EDEVICE};
  std::lock_guard<std::mutex> lock(g_scratch_m);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Status{MCC_EDEVICE};
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

int device_sms() {
  static thread_local int cached = 0;
  if (!cached) {
    int dev = 0, sms = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&sms, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        sms > 0)
      cached = sms;
    else
      cached = 256;
  }
  return cached;
}

// True if p can be dereferenced by a kernel on the current device.
bool device_visible(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
         at.devicePointer != nullptr;
}

// device_visible over many pointers: the allocation range of every pointer
// found visible is remembered, and a pointer inside a remembered range needs
// no query (a batch passes tens of pointers per instance, mostly into a few
// large allocations, and each query costs microseconds).
class VisibleRanges {
 public:
  bool check(const void* p) {
    if (!p) return false;
    const uintptr_t q = (uintptr_t)p;
    for (const auto& r : ranges_)
      if (q >= r.first && q < r.second) return true;
    if (!device_visible(p)) return false;
    void* base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && size > 0)
      ranges_.emplace_back((uintptr_t)base, (uintptr_t)base + size);
    else
      (void)hipGetLastError();
    return true;
  }

 private:
  std::vector<std::pair<uintptr_t, uintptr_t>> ranges_;
};

// Wait for the stream and surface any launch or execution error.
void sync(hipStream_t st) {
  HIPCK(hipStreamSynchronize(st));
  HIPCK(hipGetLastError());
}

template <class T>
void d2h(T* host, const T* dev, int64_t count, hipStream_t st) {
  HIPCK(hipMemcpyAsync(host, dev, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, st));
}
template <class T>
void h2d(T* dev, const T* host, int64_t count, hipStream_t st) {
  HIPCK(hipMemcpyAsync(dev, host, sizeof(T) * (size_t)count, hipMemcpyHostToDevice, st));
}

// Dense relabelling of k partitions: scan[loff[i] + x] - scan[loff[i]] is
// the id of label x of partition i, L[i] the number of distinct labels.
struct Compacted {
  const int32_t* const* dlabels = nullptr;
  int64_t* loff = nullptr;  // device, k + 1
  int32_t* scan = nullptr;  // device, loff[k] + 1
  int32_t* fmap = nullptr;  // device, loff[k] + 1: id of raw label x at loff[i] + x
  int32_t* L = nullptr;     // device, k: dense label count per partition
  std::vector<int32_t> Lh;  // host copy
  int64_t max_span = 0;     // largest maxlab + 1
};

// Everything the passes need, built from the partitions and an initial
// consensus.
struct Solve {
  int64_t n = 0;
  int32_t k = 0;
  int32_t K0 = 0;
  Compacted lab;
  int32_t* C = nullptr;
  int32_t* rawid = nullptr;
  int32_t* Lvm = nullptr;
  int32_t* s = nullptr;
  Tables t{};
  int32_t maxL = 0;        // largest label id bound of the final tables
  int64_t total = 0;       // table cells
  int64_t* acc = nullptr;  // sum s^2, sum |P_il|^2, sum N^2
  uint8_t* rdist = nullptr;  // hashed rows: distinct label ids per vertex
};

// Largest cluster count for which labels are aligned to clusters.
constexpr int32_t kAlignMaxClusters = 1 << 16;

// Largest dense table (cells) a solve may choose.  Dense tables are kept
// while they stay within 16 n k cells (or 2^24); when the clusters can be
// aligned with the labels, up to 2^30 cells (4 GiB of blocked counts): the
// aligned interleaved layout puts the counts a vertex reads for one
// candidate in one or two lines however large the table is, where a hashed
// table spreads them over k lines.  Alignment gives every partition at
// least K0 label ids, and its table is kept only within about twice the
// blocked one, so it needs K0 k <= 2 sum_i L_i (not so from singletons).
constexpr int64_t kDenseAlignedMax = (int64_t)1 << 30;

int64_t dense_cells_max(int64_t n, int32_t k, int64_t K0, int64_t sumL, bool want_rows) {
  int64_t lim = std::max<int64_t>((int64_t)1 << 24, 16 * n * (int64_t)k);
  if (want_rows && K0 <= kAlignMaxClusters && K0 * k <= 2 * sumL)
    lim = std::max(lim, kDenseAlignedMax);
  return std::min(lim, kMaxTableEntries);
}

// Blocked tables for the current label ids: allocation, zero fill, build.
Tables blocked_tables(Arena& ar, const Solve& S, const int32_t* Ldev,
                      const std::vector<int32_t>& Lh, hipStream_t st, int64_t* total) {
  const int32_t k = S.k;
  std::vector<int64_t> toff(k + 1, 0);
  for (int i = 0; i < k; ++i) toff[i + 1] = toff[i] + (int64_t)S.K0 * Lh[i];
  if (toff[k] > kMaxTableEntries) throw Status{MCC_ENOTSUP};
  int64_t* dtoff = ar.get<int64_t>(k + 1);
  h2d(dtoff, ar.host(toff), k + 1, st);
  int32_t* N = ar.get<int32_t>(toff[k]);
  launch_fill_i32(N, toff[k], 0, st);
  *total = toff[k];
  Tables t{};
  t.N = N;
  t.toff = dtoff;
  t.L = Ldev;
  t.Lmax = 0;
  t.k = k;
  t.interleaved = 0;
  return t;
}

// Stage 1: label ranges, optional init-range and CSR checks.
void compact_labels(Arena& ar, const std::vector<const int32_t*>& hptrs, int64_t n,
                    Compacted* out, int32_t* err_dev, hipStream_t st, int32_t* host_err,
                    std::vector<int32_t>* maxlab_host) {
  const int32_t k = (int32_t)hptrs.size();
  const int32_t** dl = ar.get<const int32_t*>(k);
  h2d(dl, ar.host(hptrs), k, st);
  int32_t* maxlab = ar.get<int32_t>(k);
  launch_fill_i32(maxlab, k, -1, st);
  launch_label_max(dl, k, n, maxlab, err_dev, st);
  maxlab_host->assign(k, -1);
  d2h(maxlab_host->data(), maxlab, k, st);
  d2h(host_err, err_dev, 1, st);
  out->dlabels = dl;
}

void compact_labels_finish(Arena& ar, int64_t n, int32_t k, const std::vector<int32_t>& maxlab,
                           Compacted* out, hipStream_t st) {
  std::vector<int64_t> loff(k + 1, 0);
  for (int i = 0; i < k; ++i) loff[i + 1] = loff[i] + (int64_t)maxlab[i] + 1;
  if (loff[k] > kMaxLabelFlags) throw Status{MCC_ENOTSUP};
  out->loff = ar.get<int64_t>(k + 1);
  h2d(out->loff, ar.host(loff), k + 1, st);
  int32_t* flags = ar.get<int32_t>(loff[k] + 1);
  launch_fill_i32(flags, loff[k] + 1, 0, st);
  launch_label_mark(out->dlabels, k, n, out->loff, flags, st);
  out->scan = ar.get<int32_t>(loff[k] + 1);
  int32_t* tmp = ar.get<int32_t>(scan_tmp_elems(loff[k]));
  launch_scan(flags, out->scan, loff[k], tmp, st);
  out->L = ar.get<int32_t>(k);
  launch_label_counts(out->scan, out->loff, k, out->L, st);
  out->max_span = 1;
  for (int i = 0; i < k; ++i) out->max_span = std::max<int64_t>(out->max_span, loff[i + 1] - loff[i]);
  out->fmap = ar.get<int32_t>(loff[k] + 1);
  launch_label_ids(out->scan, out->loff, k, out->max_span, out->fmap, st);
}

// Hashed layouts: the reference-aligned alignment is run when partition 0
// has at most kAlignMaxClusters labels and its blocked table against the
// other partitions stays within kRowsAlignCells counts.
constexpr int64_t kRowsAlignCells = (int64_t)1 << 27;
// Hashed rows: clusters up to this size are scored from member rows (a
// row-table probe costs about as many lines as two member rows).
constexpr int32_t kRowsMemberMax = 2;

// Choices a caller may force (results do not depend on them).
constexpr uint32_t kHashForce = 1;  // hashed tables even where dense ones fit
constexpr uint32_t kHashRows = 2;   // hashed rows whenever their indices fit
constexpr uint32_t kHashKeys = 4;   // hashed keys, no alignment

// Label ids of every partition aligned to partition 0's: the alignment of
// the interleaved layout, with partition 0's labels in the place of the
// clusters (its table is counted on a sample of the vertices; any injective
// relabelling is exact).  Partition 0's labels that the sample holds keep
// their ids.  Rewrites fmap; *L2 (device) and L2h get the new id bounds.
void align_to_reference(Arena& ar, Solve* S, int32_t maxL, int64_t sumL, int32_t** L2,
                        std::vector<int32_t>* L2h, hipStream_t st) {
  const int32_t k = S->k;
  const int64_t n = S->n;
  const std::vector<int32_t>& Lh = S->lab.Lh;
  const int32_t L0 = Lh[0];
  int32_t* Cref = ar.get<int32_t>(n);
  launch_ref_labels(S->lab.dlabels, S->lab.loff, S->lab.fmap, n, Cref, st);
  std::vector<int64_t> toff(k + 1, 0), poff(k + 1, 0);
  for (int i = 0; i < k; ++i) {
    toff[i + 1] = toff[i] + (int64_t)L0 * Lh[i];
    poff[i + 1] = poff[i] + Lh[i];
  }
  int64_t* dtoff = ar.get<int64_t>(k + 1);
  h2d(dtoff, ar.host(toff), k + 1, st);
  int64_t* dpoff = ar.get<int64_t>(k + 1);
  h2d(dpoff, ar.host(poff), k + 1, st);
  Tables bt{};
  bt.N = ar.get<int32_t>(toff[k]);
  launch_fill_i32(bt.N, toff[k], 0, st);
  bt.toff = dtoff;
  bt.L = S->lab.L;
  bt.k = k;
  const int64_t stride = std::max<int64_t>(1, n / (1 << 18));
  launch_build(Cref, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, L0, maxL, bt, st, stride);
  uint64_t* win = ar.get<uint64_t>((int64_t)k * L0);
  int32_t* home = ar.get<int32_t>(sumL);
  uint64_t* key = ar.get<uint64_t>(sumL);
  int32_t* extra = ar.get<int32_t>(sumL + 1);
  int32_t* rank = ar.get<int32_t>(sumL + 1);
  int32_t* tmp = ar.get<int32_t>(scan_tmp_elems(sumL));
  int32_t* amap = ar.get<int32_t>(sumL);
  *L2 = ar.get<int32_t>(k);
  launch_align(bt, k, L0, maxL, dpoff, sumL, win, home, key, extra, rank, tmp, amap, *L2, st);
  launch_fmap_update(S->lab.scan, S->lab.loff, dpoff, amap, k, S->lab.max_span, S->lab.fmap, st);
  L2h->assign(k, 0);
  d2h(L2h->data(), *L2, k, st);
  sync(st);
}

// The full setup: compaction of labels and clusters, tables, initial
// objective.  `init` null means singletons.  `want_rows` builds the
// vertex-major label rows the passes read.  hash_mode: kHash* bits.
void build_solve(Arena& ar, const std::vector<const int32_t*>& hptrs, int64_t n,
                 const int32_t* init, bool want_rows, const mcc_csr* g_validate, Solve* S,
                 hipStream_t st, uint32_t hash_mode = 0) {
  const int32_t k = (int32_t)hptrs.size();
  S->n = n;
  S->k = k;
  int32_t* err = ar.get<int32_t>(1);
  launch_fill_i32(err, 1, 0, st);
  int32_t* cflags = nullptr;
  if (init) {
    cflags = ar.get<int32_t>(n + 1);
    launch_fill_i32(cflags, n + 1, 0, st);
    launch_cluster_mark(init, n, cflags, err, st);
  }
  if (g_validate)
    launch_validate_csr(g_validate->row_ptr, g_validate->col, n, g_validate->nnz, err, st);
  int32_t herr = 0;
  std::vector<int32_t> maxlab;
  compact_labels(ar, hptrs, n, &S->lab, err, st, &herr, &maxlab);
  sync(st);
  if (herr & kErrGraph) throw Status{MCC_EGRAPH};
  if (herr & (kErrNegLabel | kErrInitRange)) throw Status{MCC_EINVAL};
  compact_labels_finish(ar, n, k, maxlab, &S->lab, st);
  int32_t* cmap = nullptr;
  if (init) {
    cmap = ar.get<int32_t>(n + 1);
    int32_t* tmp = ar.get<int32_t>(scan_tmp_elems(n));
    launch_scan(cflags, cmap, n, tmp, st);
  }
  S->lab.Lh.assign(k, 0);
  d2h(S->lab.Lh.data(), S->lab.L, k, st);
  int32_t K0 = (int32_t)n;
  if (init) d2h(&K0, cmap + n, 1, st);
  sync(st);
  S->K0 = K0;

  S->C = ar.get<int32_t>(n);
  S->rawid = ar.get<int32_t>(K0);
  if (init) {
    launch_cluster_assign(init, n, cmap, S->C, S->rawid, st);
  } else {
    launch_iota(S->C, n, st);
    launch_iota(S->rawid, n, st);
  }
  S->s = ar.get<int32_t>(K0);
  launch_fill_i32(S->s, K0, 0, st);
  launch_sizes(S->C, n, K0, S->s, st);

  const std::vector<int32_t>& Lh = S->lab.Lh;
  int32_t maxL = 1;
  int64_t sumL = 0;
  for (int i = 0; i < k; ++i) {
    maxL = std::max(maxL, Lh[i]);
    sumL += Lh[i];
  }
  // Hashed tables when the dense ones would not fit, or would be far larger
  // than the n k keys a hashed table holds at most (unless they can be
  // aligned: dense_cells_max).
  const int64_t dense = (int64_t)K0 * sumL;
  if ((hash_mode & kHashForce) || dense > dense_cells_max(n, k, K0, sumL, want_rows)) {
    int bits = 12;
    while (((int64_t)1 << bits) < 4 * n * (int64_t)k) ++bits;
    const int64_t slots = (int64_t)1 << bits;
    if (slots > kMaxHashSlots) throw Status{MCC_ENOTSUP};
    Tables t{};
    t.k = k;
    t.hashed = 1;
    int32_t* hc = ar.get<int32_t>(2);
    launch_fill_i32(hc, 2, 0, st);
    t.hocc = hc;
    t.herr = hc + 1;
    // Hashed rows when the aligned labels give few rows: every live row
    // (x, l) holds a label id l of one of x's members, so no clustering has
    // more live rows than the singletons' T0 (the sum over vertices of
    // their distinct ids), and a pass adds at most T0 more, so more than
    // 2 T0 rows always leave an empty one (rebuilds keep the table about
    // half full in practice).  Taken when that table is no larger than the
    // key table and its cell indices fit 31 bits.
    std::vector<int32_t> Lk = Lh;  // label id bounds of the table's keys
    const int32_t* Lk_dev = S->lab.L;
    bool rows = false;
    if (want_rows && !(hash_mode & kHashKeys) && Lh[0] <= kAlignMaxClusters &&
        (int64_t)Lh[0] * sumL <= kRowsAlignCells) {
      int32_t* L2 = nullptr;
      std::vector<int32_t> L2h;
      align_to_reference(ar, S, maxL, sumL, &L2, &L2h, st);
      Lk = L2h;
      Lk_dev = L2;
      S->Lvm = ar.get<int32_t>(n * k);
      launch_label_transpose(S->lab.dlabels, k, n, S->lab.loff, S->lab.fmap, S->Lvm, st);
      uint8_t* rdist = ar.get<uint8_t>(n);
      int64_t* tot = ar.get<int64_t>(1);
      launch_fill_u64(reinterpret_cast<uint64_t*>(tot), 1, 0ull, st);
      launch_row_distinct(S->Lvm, n, k, rdist, tot, st);
      int64_t T0 = 0;
      d2h(&T0, tot, 1, st);
      sync(st);
      int rbits = 12;
      while (((int64_t)1 << rbits) <= 2 * T0) ++rbits;
      const int64_t R = (int64_t)1 << rbits;
      const bool fits = R * k + 2 * (int64_t)K0 < ((int64_t)1 << 31);
      const bool smaller = R * (8 + 4 * (int64_t)k) <= 16 * slots;
      if (fits && (smaller || (hash_mode & kHashRows))) {
        rows = true;
        t.rows = 1;
        t.rkeys = ar.get<uint64_t>(R);
        t.N = ar.get<int32_t>(R * k);
        launch_fill_i32(t.N, R * k, 0, st);
        t.hshift = 64 - rbits;
        t.hmask = (uint64_t)R - 1;
        S->rdist = rdist;
        S->total = R * k;
      }
    }
    int32_t maxLk = 1;
    std::vector<int64_t> poff(k + 1, 0);
    for (int i = 0; i < k; ++i) {
      poff[i + 1] = poff[i] + Lk[i];
      maxLk = std::max(maxLk, Lk[i]);
    }
    int64_t* dpoff = ar.get<int64_t>(k + 1);
    h2d(dpoff, ar.host(poff), k + 1, st);
    t.toff = dpoff;
    t.L = Lk_dev;
    if (!rows) {
      t.N = ar.get<int32_t>(4 * slots);
      t.hshift = 64 - bits;
      t.hmask = (uint64_t)slots - 1;
      S->total = slots;
    }
    launch_hash_clear(t, st);
    if (rows && K0 == n)  // one vertex a cluster: every row has one owner
      launch_build_rows_single(S->C, S->Lvm, n, k, t, st);
    else if (rows)  // from the vertex-major rows: a vertex's k updates share few rows
      launch_build_rows(S->C, S->Lvm, n, k, t, st);
    else
      launch_build(S->C, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, K0, maxLk, t, st);
    S->t = t;
    S->maxL = maxLk;
    if (want_rows && !S->Lvm) {
      S->Lvm = ar.get<int32_t>(n * k);
      launch_label_transpose(S->lab.dlabels, k, n, S->lab.loff, S->lab.fmap, S->Lvm, st);
    }
    S->acc = ar.get<int64_t>(3);
    launch_fill_u64(reinterpret_cast<uint64_t*>(S->acc), 3, 0ull, st);
    int32_t* hist = ar.get<int32_t>(poff[k]);
    launch_objective0_hashed(t, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, K0, S->s,
                             poff[k], hist, K0 == n, S->acc, st);
    return;
  }
  // Blocked tables with dense label ids: the final tables when the labels
  // are not aligned; otherwise first built from a sample of the vertices as
  // the source of the alignment (any injective relabelling is exact, so the
  // sample only steers the layout).
  int64_t total = 0;
  Tables bt = blocked_tables(ar, *S, S->lab.L, Lh, st, &total);
  const bool try_align = want_rows && K0 <= kAlignMaxClusters;
  const int64_t stride = try_align ? std::max<int64_t>(1, n / (1 << 18)) : 1;
  launch_build(S->C, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, K0, maxL, bt, st, stride);
  S->t = bt;
  S->maxL = maxL;
  S->total = total;
  bool aligned = false;
  std::vector<int32_t> Lfinal = Lh;  // label ids per partition in the final layout

  if (try_align) {
    std::vector<int64_t> poff(k + 1, 0);
    for (int i = 0; i < k; ++i) poff[i + 1] = poff[i] + Lh[i];
    int64_t* dpoff = ar.get<int64_t>(k + 1);
    h2d(dpoff, ar.host(poff), k + 1, st);
    uint64_t* win = ar.get<uint64_t>((int64_t)k * K0);
    int32_t* home = ar.get<int32_t>(sumL);
    uint64_t* key = ar.get<uint64_t>(sumL);
    int32_t* extra = ar.get<int32_t>(sumL + 1);
    int32_t* rank = ar.get<int32_t>(sumL + 1);
    int32_t* tmp = ar.get<int32_t>(scan_tmp_elems(sumL));
    int32_t* amap = ar.get<int32_t>(sumL);
    int32_t* L2 = ar.get<int32_t>(k);
    launch_align(bt, k, K0, maxL, dpoff, sumL, win, home, key, extra, rank, tmp, amap, L2, st);
    std::vector<int32_t> L2h(k, 0);
    d2h(L2h.data(), L2, k, st);
    sync(st);
    int32_t Lmax = 1;
    for (int i = 0; i < k; ++i) Lmax = std::max(Lmax, L2h[i]);
    const int64_t cells = (int64_t)K0 * Lmax * k;
    if (cells <= kMaxTableEntries && cells <= 2 * total + ((int64_t)1 << 20) &&
        cells + 2 * (int64_t)K0 < ((int64_t)1 << 31)) {
      launch_fmap_update(S->lab.scan, S->lab.loff, dpoff, amap, k, S->lab.max_span,
                         S->lab.fmap, st);
      Tables it{};
      it.N = ar.get<int32_t>(cells);
      launch_fill_i32(it.N, cells, 0, st);
      it.toff = nullptr;
      it.L = L2;
      it.Lmax = Lmax;
      it.k = k;
      it.interleaved = 1;
      launch_build(S->C, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, K0, Lmax, it, st);
      S->t = it;
      S->maxL = Lmax;
      S->total = cells;
      aligned = true;
      Lfinal = L2h;
    }
  }
  if (try_align && !aligned && stride > 1) {  // sampled blocked tables: count them all
    launch_fill_i32(bt.N, total, 0, st);
    launch_build(S->C, S->lab.dlabels, S->lab.loff, S->lab.fmap, n, k, K0, maxL, bt, st, 1);
  }
  if (want_rows) {
    S->Lvm = ar.get<int32_t>(n * k);
    launch_label_transpose(S->lab.dlabels, k, n, S->lab.loff, S->lab.fmap, S->Lvm, st);
  }
  S->acc = ar.get<int64_t>(3);
  launch_fill_u64(reinterpret_cast<uint64_t*>(S->acc), 3, 0ull, st);
  std::vector<int64_t> lpoff(k + 1, 0);
  for (int i = 0; i < k; ++i) lpoff[i + 1] = lpoff[i] + Lfinal[i];
  LabelHist lh{};
  lh.dlabels = S->lab.dlabels;
  lh.loff = S->lab.loff;
  lh.fmap = S->lab.fmap;
  int64_t* dlpoff = ar.get<int64_t>(k + 1);
  h2d(dlpoff, ar.host(lpoff), k + 1, st);
  lh.lpoff = dlpoff;
  lh.total_labels = lpoff[k];
  lh.hist = ar.get<int32_t>(lpoff[k]);
  launch_objective0(S->t, k, K0, S->maxL, S->s, S->total, lh, S->C, S->Lvm, n, S->acc, st);
}

int translate(const std::exception_ptr& ep) {
  try {
    std::rethrow_exception(ep);
  } catch (const Status& s) {
    return s.code;
  } catch (const NoMem&) {
    return MCC_ENOMEM;
  } catch (const HipError&) {
    return MCC_EDEVICE;
  } catch (...) {
    g_hip_error = "unexpected host exception";
    return MCC_EDEVICE;
  }
}

bool labels_ok(const int32_t* const* labels, int32_t k) {
  if (!labels) return false;
  for (int i = 0; i < k; ++i)
    if (!device_visible(labels[i])) return false;
  return true;
}

}  // namespace

extern "C" {

const char* mcc_strerror(int code) {
  switch (code) {
    case MCC_OK: return "success";
    case MCC_EINVAL: return "invalid argument";
    case MCC_EGRAPH: return "invalid CSR graph";
    case MCC_ENOMEM: return "out of device memory";
    case MCC_EDEVICE: return g_hip_error.empty() ? "HIP runtime error" : g_hip_error.c_str();
    case MCC_ENOTSUP: return "instance exceeds the supported table size";
    case MCC_ESCRATCH:
      return "instance needs more workspace than the no-allocation scratch array holds";
    default: return "unknown error code";
  }
}

}  // extern "C"

namespace {

// One solve.  noalloc: the workspace is the device's scratch array instead
// of the cached chunks (nothing is allocated).
int consensus_impl(const mcc_csr* g, const int32_t* const* labels, int32_t k,
                   const int32_t* init, int32_t* out, mcc_stats* stats, bool noalloc) {
  if (!g || k < 1 || g->n < 0 || g->nnz < 0) return MCC_EINVAL;
  const int64_t n = g->n;
  const int32_t max_rounds = stats && stats->max_rounds > 0 ? stats->max_rounds : 1000;
  const uint32_t flags = stats ? stats->flags : 0u;
  const int lanes_req = stats ? stats->lanes : 0;
  if (stats && stats->max_rounds < 0) return MCC_EINVAL;
  if (lanes_req != 0 && !score_lanes_ok(lanes_req)) return MCC_EINVAL;
  if ((flags & MCC_F_TRACE) && !stats->trace) return MCC_EINVAL;
  if ((int64_t)k * n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  if (!labels) return MCC_EINVAL;
  if (g->nnz >= ((int64_t)1 << 31) - 1) return MCC_ENOTSUP;  // 32-bit arc positions
  if (stats) {
    stats->passes = stats->converged = stats->fallback_rounds = stats->clusters = 0;
    stats->moves = stats->candidate_evals = stats->objective_init = stats->objective = 0;
    stats->ms_total = stats->ms_passes = stats->ms_score = 0.f;
    stats->boundary = 0;
    stats->lanes_used = 0;
    stats->tables = 0;
    stats->skipped_evals = 0;
    stats->workspace_bytes = 0;
  }
  if (n == 0) {
    if (stats) {
      stats->passes = 1;
      stats->converged = 1;
      if (flags & MCC_F_TRACE) memset(stats->trace, 0, 4 * sizeof(int64_t));
    }
    return MCC_OK;
  }
  if (!device_visible(g->row_ptr) || (g->nnz > 0 && !device_visible(g->col)) ||
      !device_visible(out) || (init && !device_visible(init)) || !labels_ok(labels, k))
    return MCC_EINVAL;

  hipStream_t st = stats ? (hipStream_t)stats->stream : nullptr;
  // the label rows and per-vertex state alone must fit the scratch array
  if (noalloc && (uint64_t)(4 * n * (int64_t)k + 48 * n) > kScratchBytes) return MCC_ESCRATCH;
  try {
    Arena ar(st, noalloc ? scratch_address() : nullptr, kScratchBytes);
    hipEvent_t e0, e1, e2, e3;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    HIPCK(hipEventCreate(&e2));
    HIPCK(hipEventCreate(&e3));
    struct Ev {
      hipEvent_t* e;
      ~Ev() {
        for (int j = 0; j < 4; ++j) (void)hipEventDestroy(e[j]);
      }
    };
    hipEvent_t evs[4] = {e0, e1, e2, e3};
    Ev guard{evs};
    HIPCK(hipEventRecord(e0, st));

    std::vector<const int32_t*> hptrs(labels, labels + k);
    Solve S;
    build_solve(ar, hptrs, n, init, true, (flags & MCC_F_VALIDATE) ? g : nullptr, &S, st,
                ((flags & MCC_F_HASH_TABLES) ? kHashForce : 0u) |
                    ((flags & MCC_F_HASH_ROWS) ? kHashRows : 0u) |
                    ((flags & MCC_F_HASH_KEYS) ? kHashKeys : 0u));

    int64_t* dtrace = nullptr;
    if (flags & MCC_F_TRACE) dtrace = ar.get<int64_t>((int64_t)max_rounds * 4);
    Ctl* ctl = ar.get<Ctl>(1);
    launch_ctl_init(ctl, S.acc, k, max_rounds, dtrace, st);
    uint64_t* owner = ar.get<uint64_t>(S.K0);
    launch_fill_u64(owner, S.K0, ~0ull, st);
    int32_t* prop = ar.get<int32_t>(n);
    int64_t* dprop = ar.get<int64_t>(n);
    int32_t* heavy = ar.get<int32_t>(n);
    // arc clusters and in-arc lists, on request
    const int64_t nnz = g->nnz;
    int32_t* in_ptr = nullptr;
    int32_t* in_pos = nullptr;
    int32_t* ac = nullptr;
    if (flags & MCC_F_ARC_CACHE) {
      in_ptr = ar.get<int32_t>(n + 1);
      int32_t* indeg = ar.get<int32_t>(n + 1);
      launch_fill_i32(indeg, n + 1, 0, st);
      launch_in_degree(g->col, nnz, indeg, st);
      int32_t* stmp = ar.get<int32_t>(scan_tmp_elems(n));
      launch_scan(indeg, in_ptr, n, stmp, st);
      launch_copy_i32(in_ptr, indeg, n, st);  // cursors
      in_pos = ar.get<int32_t>(nnz);
      launch_in_fill(g->col, nnz, indeg, in_pos, st);
      ac = ar.get<int32_t>(nnz);
      launch_arc_clusters(g->col, nnz, S.C, ac, st);
    }

    PassArgs a{};
    a.ctl = ctl;
    a.pc = ar.get<int64_t>(kPassCounters * kCounterStride);
    a.plist = ar.get<int32_t>(n);
    if (!S.t.hashed) {  // histogram apply when a partition's slice fits in LDS
      const int64_t slice = (int64_t)S.K0 * S.maxL + 2 * (int64_t)S.K0;
      if (4 * slice <= kDeltaLdsMax) {
        a.delta_lds = (int32_t)(4 * slice);
        a.delta_slices = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, n / 2048));
      }
    }
    launch_fill_u64(reinterpret_cast<uint64_t*>(a.pc), kPassCounters * kCounterStride, 0ull, st);
    a.n = n;
    a.k = k;
    a.literal = (flags & MCC_F_LITERAL) ? 1 : 0;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.C = S.C;
    a.Lvm = S.Lvm;
    a.t = S.t;
    a.s = S.s;
    a.prop = prop;
    a.dprop = dprop;
    a.owner = owner;
    a.heavy = heavy;
    a.ac = ac;
    a.in_ptr = in_ptr;
    a.in_pos = in_pos;
    a.cells = S.total;
    a.nnz = nnz;
    a.arcs_aligned = ((uintptr_t)g->col & 15) == 0 ? 1 : 0;  // ac comes from the arena (aligned)
    if ((flags & MCC_F_SYMMETRIC) && (flags & MCC_F_VALIDATE)) {
      int32_t* serr = ar.get<int32_t>(1);
      launch_fill_i32(serr, 1, 0, st);
      launch_check_symmetric(g->row_ptr, g->col, n, serr, st);
      int32_t hs = 0;
      d2h(&hs, serr, 1, st);
      sync(st);
      if (hs) throw Status{MCC_EGRAPH};
    }
    a.hflag = S.t.hashed ? ar.get<int32_t>(1) : nullptr;
    a.rdist = S.t.rows ? S.rdist : nullptr;
    a.K0 = S.K0;
    if (S.t.hashed) {
      a.mstart = ar.get<int32_t>((int64_t)S.K0 + 1);
      a.mcnt = ar.get<int32_t>(S.K0);
      a.members = ar.get<int32_t>(n);
      a.mscan_tmp = ar.get<int32_t>(scan_tmp_elems(S.K0));
      a.msum_max = S.t.rows ? kRowsMemberMax : kMemberSumMax;
    }
    a.cn_bytes = S.K0 <= 256 ? 1 : (S.K0 <= 65536 ? 2 : 4);
    if (a.cn_bytes == 4) {
      a.Cn = S.C;
    } else {
      a.Cn = ar.get<uint8_t>(n * a.cn_bytes);
      launch_narrow(S.C, a.Cn, a.cn_bytes, n, st);
    }
    // 32-bit update keys: cells, cluster sizes, per-cluster move counts
    if (S.total + 2 * (int64_t)S.K0 >= ((int64_t)1 << 31)) throw Status{MCC_ENOTSUP};

    // the tiled scorer packs cluster ids in 24 bits
    const int lanes = (lanes_req == 0 && S.K0 >= (1 << 24)) ? 64 : lanes_req;
    if ((flags & MCC_F_SYMMETRIC) && lanes == 0) {  // candidate sets carried over
      a.dirty = ar.get<int32_t>(n);
      a.cnum = ar.get<int32_t>(n);
      a.ccache = ar.get<int32_t>(n * kCacheCand);
      launch_fill_i32(a.dirty, n, 1, st);
      launch_fill_i32(a.cnum, n, -1, st);
      a.slack = ar.get<int32_t>(n);
      a.churn = ar.get<int32_t>(2 * (int64_t)S.K0);
      a.st = ar.get<int32_t>(n);
      a.rlist = ar.get<int32_t>(n);
      a.sparse_max = (int32_t)std::max<int64_t>(1, n / 8);
      // the cached candidate rows are read as 16-byte vectors
      launch_fill_i32(a.slack, n, -1, st);
      launch_fill_i32(a.churn, 2 * (int64_t)S.K0, 0, st);
    }
    const int sms = device_sms();
    const int64_t blocks_needed =
        lanes ? (n * lanes + kBlock - 1) / kBlock : (n + kBlock - 1) / kBlock;
    const int grid_score = (int)std::max<int64_t>(1, std::min<int64_t>(blocks_needed, sms * 8));
    const int grid_apply =
        (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, sms * 4));

    const bool profile = (flags & MCC_F_PROFILE) != 0;
    std::vector<hipEvent_t> pev;  // begin/end of every enqueued scoring kernel
    struct EvList {
      std::vector<hipEvent_t>* v;
      ~EvList() {
        for (hipEvent_t e : *v) (void)hipEventDestroy(e);
      }
    } pev_guard{&pev};

    HIPCK(hipEventRecord(e1, st));
    Ctl hc;
    memset(&hc, 0, sizeof hc);
    int enqueued = 0, chunk = 2;
    while (enqueued < max_rounds) {
      const int todo = std::min(chunk, max_rounds - enqueued);
      for (int j = 0; j < todo; ++j) {
        hipEvent_t b = nullptr, e = nullptr;
        if (profile) {
          HIPCK(hipEventCreate(&b));
          pev.push_back(b);
          HIPCK(hipEventCreate(&e));
          pev.push_back(e);
        }
        enqueue_pass(a, lanes, grid_score, grid_apply, st, b, e);
      }
      enqueued += todo;
      d2h(&hc, ctl, 1, st);
      sync(st);
      if (hc.done) break;
      chunk = std::min(chunk * 2, 16);
    }
    HIPCK(hipEventRecord(e2, st));

    launch_finish(S.C, S.rawid, n, out, st);
    int32_t* ncl = ar.get<int32_t>(1);
    launch_fill_i32(ncl, 1, 0, st);
    launch_count_nonzero(S.s, S.K0, ncl, st);
    int32_t clusters = 0;
    d2h(&clusters, ncl, 1, st);
    d2h(&hc, ctl, 1, st);
    int64_t acc[3];
    d2h(acc, S.acc, 3, st);
    int32_t hash_err = 0;
    if (S.t.hashed) d2h(&hash_err, S.t.herr, 1, st);
    HIPCK(hipEventRecord(e3, st));
    sync(st);
    if (hash_err) throw Status{MCC_ENOMEM};  // cannot happen: the table stays half empty
    if (flags & MCC_F_TRACE) {
      memset(stats->trace, 0, sizeof(int64_t) * 4 * (size_t)max_rounds);
      d2h(stats->trace, dtrace, (int64_t)4 * hc.passes, st);
      sync(st);
    }
    if (stats) {
      stats->passes = hc.passes;
      stats->converged = hc.converged;
      stats->fallback_rounds = hc.fallback_rounds;
      stats->clusters = clusters;
      stats->moves = hc.moves;
      stats->candidate_evals = hc.evals;
      stats->skipped_evals = hc.skipped;
      stats->workspace_bytes = (int64_t)ar.bytes_used();
      stats->objective_init = (int64_t)k * acc[0] + acc[1] - 2 * acc[2];
      stats->objective = hc.O;
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, e0, e3));
      stats->ms_total = ms;
      HIPCK(hipEventElapsedTime(&ms, e1, e2));
      stats->ms_passes = ms;
      stats->boundary = hc.boundary;
      stats->lanes_used = lanes;
      stats->tables = S.t.hashed ? (S.t.rows ? 3 : 2) : (S.t.interleaved ? 1 : 0);
      if (profile) {
        float tot = 0.f;
        for (int j = 0; j < hc.passes && 2 * j + 1 < (int)pev.size(); ++j) {
          HIPCK(hipEventElapsedTime(&ms, pev[2 * j], pev[2 * j + 1]));
          tot += ms;
        }
        stats->ms_score = tot;
      }
    }
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

}  // namespace

extern "C" {

int mcc_consensus(const mcc_csr* g, const int32_t* const* labels, int32_t k, const int32_t* init,
                  int32_t* out, mcc_stats* stats) {
  return consensus_impl(g, labels, k, init, out, stats, false);
}

int mcc_consensus_noalloc(const mcc_csr* g, const int32_t* const* labels, int32_t k,
                          const int32_t* init, int32_t* out, mcc_stats* stats) {
  return consensus_impl(g, labels, k, init, out, stats, true);
}

int mcc_objective(const int32_t* c, const int32_t* const* labels, int32_t k, int64_t n,
                  int64_t* result, void* stream) {
  if (!result || k < 1 || n < 0) return MCC_EINVAL;
  if ((int64_t)k * n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  if (n == 0) {
    *result = 0;
    return MCC_OK;
  }
  if (!device_visible(c) || !labels_ok(labels, k)) return MCC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    Arena ar(st);
    std::vector<const int32_t*> hptrs(labels, labels + k);
    Solve S;
    build_solve(ar, hptrs, n, c, false, nullptr, &S, st);
    int64_t acc[3];
    d2h(acc, S.acc, 3, st);
    sync(st);
    *result = (int64_t)k * acc[0] + acc[1] - 2 * acc[2];
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

int mcc_mirkin(const int32_t* a, const int32_t* b, int64_t n, int64_t* result, void* stream) {
  if (!result || n < 0 || n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  if (n == 0) {
    *result = 0;
    return MCC_OK;
  }
  if (!device_visible(a) || !device_visible(b)) return MCC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    Arena ar(st);
    // dense ids of a (in [0, n)) serve as the consensus, b as the single
    // partition: the objective with k = 1 is Mirkin(a, b)
    std::vector<const int32_t*> pa{a};
    Compacted ca;
    int32_t* err = ar.get<int32_t>(1);
    launch_fill_i32(err, 1, 0, st);
    int32_t herr = 0;
    std::vector<int32_t> maxlab;
    compact_labels(ar, pa, n, &ca, err, st, &herr, &maxlab);
    sync(st);
    if (herr & kErrNegLabel) return MCC_EINVAL;
    compact_labels_finish(ar, n, 1, maxlab, &ca, st);
    int32_t* da = ar.get<int32_t>(n);
    launch_dense_map(a, n, ca.scan, da, st);
    std::vector<const int32_t*> pb{b};
    Solve S;
    build_solve(ar, pb, n, da, false, nullptr, &S, st);
    int64_t acc[3];
    d2h(acc, S.acc, 3, st);
    sync(st);
    *result = acc[0] + acc[1] - 2 * acc[2];
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

int mcc_canonicalize(const int32_t* in, int32_t* out, int64_t n, int32_t* clusters,
                     void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  if (n == 0) {
    if (clusters) *clusters = 0;
    return MCC_OK;
  }
  if (!device_visible(in) || !device_visible(out)) return MCC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    Arena ar(st);
    int32_t* err = ar.get<int32_t>(1);
    launch_fill_i32(err, 1, 0, st);
    int32_t* cflags = ar.get<int32_t>(n + 1);
    launch_fill_i32(cflags, n + 1, 0, st);
    launch_cluster_mark(in, n, cflags, err, st);  // range check
    int32_t herr = 0;
    d2h(&herr, err, 1, st);
    sync(st);
    if (herr) return MCC_EINVAL;
    int32_t* first = ar.get<int32_t>(n);
    launch_fill_i32(first, n, 0x7fffffff, st);
    launch_first_occurrence(in, n, first, st);
    int32_t* fl = ar.get<int32_t>(n + 1);
    launch_first_flags(in, n, first, fl, st);
    int32_t* rank = ar.get<int32_t>(n + 1);
    int32_t* tmp = ar.get<int32_t>(scan_tmp_elems(n));
    launch_scan(fl, rank, n, tmp, st);
    launch_canonical_write(in, n, first, rank, out, st);
    int32_t total = 0;
    d2h(&total, rank + n, 1, st);
    sync(st);
    if (clusters) *clusters = total;
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

// ---------------------------------------------------------------------------
// Batched solves: host checks, launch shape, one persistent launch.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr int kTuneLanes[MCC_TUNE_LANES] = {4, 8, 16, 32, 64};
constexpr int64_t kCellsCapMin = (int64_t)1 << 16;
constexpr int64_t kCellsCapMax = (int64_t)1 << 23;

int n_log2_of(int64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

int k_class_of(int32_t k) { return k <= 8 ? 0 : k <= 16 ? 1 : k <= 32 ? 2 : k <= 64 ? 3 : 4; }

// Lanes per vertex when no tune table covers an instance.  Measured on SBM
// instances with n in [200, 20000] and k in [8, 64]: more vertices in flight
// beat more lanes per vertex for every k; 4 lanes lead below about 4096
// vertices, 8 above.
int default_lanes(int64_t n) { return n < 4096 ? 4 : 8; }

// The table entry of the instance's bucket, else of the nearest n bucket
// with the same k class, else null.
const mcc_tune_entry* tune_lookup(const mcc_tune_table* t, int64_t n, int32_t k) {
  if (!t) return nullptr;
  const int nb = n_log2_of(n), kc = k_class_of(k);
  const mcc_tune_entry* best = nullptr;
  int bestd = 1 << 30;
  for (int j = 0; j < t->count && j < MCC_TUNE_MAX_BUCKETS; ++j) {
    const mcc_tune_entry& e = t->entry[j];
    if (e.k_class != kc) continue;
    const int d = std::abs(e.n_log2 - nb);
    if (d < bestd) {
      bestd = d;
      best = &e;
    }
  }
  return best;
}

int64_t pow2_ceil(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

bool problem_ok(const mcc_problem& p, bool need_out, VisibleRanges& vis) {
  const int64_t n = p.g.n;
  bool ok = p.k >= 1 && n >= 0 && p.g.nnz >= 0 && p.labels &&
            (int64_t)p.k * n < ((int64_t)1 << 31) && p.g.nnz < ((int64_t)1 << 31) - 1;
  if (ok && n > 0) {
    ok = vis.check(p.g.row_ptr) && (p.g.nnz == 0 || vis.check(p.g.col)) &&
         (!need_out || vis.check(p.out)) && (!p.init || vis.check(p.init));
    for (int i = 0; ok && i < p.k; ++i) ok = vis.check(p.labels[i]);
  }
  return ok;
}

// The persistent launch as a one-node HIP graph per (device, stream),
// instantiated once and replayed: each call sets the node's arguments and
// grid.  Its queue counter lives with it (never reset; see BatchArgs).
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  unsigned long long* queue = nullptr;
  unsigned long long qnext = 0;
};

struct GraphCache {
  std::mutex m;
  std::map<std::pair<int, hipStream_t>, BatchGraph> g;
};

GraphCache& graph_cache() {
  static GraphCache* c = new GraphCache;  // never destroyed: may outlive static teardown
  return *c;
}

void destroy_graph(BatchGraph& bg) {
  if (bg.exec) (void)hipGraphExecDestroy(bg.exec);
  if (bg.graph) (void)hipGraphDestroy(bg.graph);
  if (bg.queue) (void)hipFree(bg.queue);
  bg = BatchGraph{};
}

// Launch the persistent kernel over `ba` (ba.queue and ba.qbase are filled
// here) through the stream's graph, bracketed by the two events.
void launch_batch_graph(BatchArgs& ba, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> lock(c.m);
  BatchGraph& bg = c.g[{dev, st}];
  if (!bg.queue) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(unsigned long long));
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      throw NoMem{};
    }
    hipck(e, "hipMalloc");
    bg.queue = static_cast<unsigned long long*>(q);
    launch_fill_u64(reinterpret_cast<uint64_t*>(bg.queue), 1, 0ull, st);
    bg.qnext = 0;
  }
  ba.queue = bg.queue;
  ba.qbase = bg.qnext;
  void* args[] = {&ba};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(batch_kernel());
  kp.gridDim = dim3((unsigned)grid);
  kp.blockDim = dim3(kBlock);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  hipError_t e = hipSuccess;
  if (!bg.exec) {
    e = hipGraphCreate(&bg.graph, 0);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&bg.node, bg.graph, nullptr, 0, &kp);
    if (e == hipSuccess) e = hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0);
  } else {
    e = hipGraphExecKernelNodeSetParams(bg.exec, bg.node, &kp);
  }
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = hipGraphLaunch(bg.exec, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e != hipSuccess) {  // the counter may be out of step: start over next time
    destroy_graph(bg);
    c.g.erase({dev, st});
    HIPCK(e);
  }
  bg.qnext += (unsigned long long)ba.count + (unsigned long long)grid;
}

// Sizes of the persistent launch's workspace for a set of problems.
struct BatchSizes {
  int64_t n_max = 1;
  int32_t k_max = 1;
  int64_t slots = 1;
  int64_t labels = 0;  // label pointers
  int64_t bytes = 0;   // device bytes, allocation by allocation as the arena rounds them
};

int64_t arena_round(int64_t bytes) { return (std::max<int64_t>(bytes, 1) + 255) & ~(int64_t)255; }

BatchSizes batch_sizes(const mcc_problem* probs, const std::vector<int32_t>& ids, int32_t count,
                       int64_t cells_cap, int wgpc) {
  BatchSizes z;
  for (int32_t i : ids) {
    z.labels += probs[i].k;
    z.n_max = std::max<int64_t>(z.n_max, probs[i].g.n);
    z.k_max = std::max<int32_t>(z.k_max, probs[i].k);
  }
  z.slots = std::max<int64_t>(1, std::min<int64_t>((int64_t)ids.size(),
                                                   (int64_t)device_sms() * wgpc));
  const int64_t flag_cap = 2 * z.n_max + 1024;
  z.bytes = arena_round(8 * std::max<int64_t>(1, z.labels)) +
            4 * arena_round(4 * z.slots * z.n_max) +            // C, rawid, prop, s
            2 * arena_round(8 * z.slots * z.n_max) +            // dprop, owner
            arena_round(4 * z.slots * z.n_max * z.k_max) +      // label rows
            arena_round(4 * z.slots * cells_cap) +              // tables
            arena_round(4 * z.slots * flag_cap) +               // flags
            arena_round((int64_t)sizeof(BatchInst) * count) + arena_round(4 * (int64_t)ids.size()) +
            arena_round((int64_t)sizeof(BatchRes) * count);
  return z;
}

struct BatchRun {
  const mcc_problem* probs = nullptr;
  std::vector<int32_t> ids;      // problems to run
  std::vector<int32_t> lanes;    // per problem (indexed like probs)
  std::vector<int32_t*> outs;    // per problem: output buffer override, or null
  int wgpc = 2;
  int64_t cells_cap = 0;
  int32_t max_rounds = 1000;
  int32_t literal = 0;
};

// One persistent launch over run.ids; per-problem results land in hres
// (indexed like probs); returns the launch's time on the stream in ms.
float run_batch(const BatchRun& run, int32_t count, hipStream_t st, std::vector<BatchRes>* hres,
                int64_t* ws_bytes = nullptr) {
  Arena ar(st);  // the launch's workspace, released on return
  const mcc_problem* probs = run.probs;
  std::vector<const int32_t*> allptr;
  std::vector<BatchInst> hinst(count);
  std::vector<int64_t> loff(count, 0);
  int64_t n_max = 1;
  int32_t k_max = 1;
  for (int32_t i : run.ids) {
    loff[i] = (int64_t)allptr.size();
    for (int j = 0; j < probs[i].k; ++j) allptr.push_back(probs[i].labels[j]);
    n_max = std::max<int64_t>(n_max, probs[i].g.n);
    k_max = std::max<int32_t>(k_max, probs[i].k);
  }
  const int32_t** dptrs = ar.get<const int32_t*>((int64_t)std::max<size_t>(1, allptr.size()));
  if (!allptr.empty()) h2d(dptrs, ar.host(allptr), (int64_t)allptr.size(), st);
  for (int32_t i : run.ids) {
    const mcc_problem& p = probs[i];
    BatchInst b{};
    b.n = p.g.n;
    b.nnz = p.g.nnz;
    b.row_ptr = p.g.row_ptr;
    b.col = p.g.col;
    b.labels = dptrs + loff[i];
    b.init = p.init;
    b.out = run.outs.empty() || !run.outs[i] ? p.out : run.outs[i];
    b.k = p.k;
    b.lanes = run.lanes[i];
    hinst[i] = b;
  }
  // largest estimated work first
  std::vector<int32_t> order(run.ids);
  auto work = [&](int32_t i) { return probs[i].g.nnz + probs[i].g.n * (int64_t)probs[i].k; };
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return work(a) > work(b); });

  BatchArgs ba{};
  BatchWs& w = ba.ws;
  w.n_max = n_max;
  w.k_max = k_max;
  w.flag_cap = 2 * n_max + 1024;
  w.cells_cap = run.cells_cap;
  const int64_t slots = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)run.ids.size(), (int64_t)device_sms() * run.wgpc));
  w.C = ar.get<int32_t>(slots * n_max);
  w.rawid = ar.get<int32_t>(slots * n_max);
  w.prop = ar.get<int32_t>(slots * n_max);
  w.dprop = ar.get<int64_t>(slots * n_max);
  w.s = ar.get<int32_t>(slots * n_max);
  w.owner = ar.get<uint64_t>(slots * n_max);
  w.Lvm = ar.get<int32_t>(slots * n_max * k_max);
  w.N = ar.get<int32_t>(slots * w.cells_cap);
  w.flags = ar.get<int32_t>(slots * w.flag_cap);
  BatchInst* dinst = ar.get<BatchInst>(count);
  h2d(dinst, ar.host(hinst), count, st);
  int32_t* dorder = ar.get<int32_t>((int64_t)order.size());
  h2d(dorder, ar.host(order), (int64_t)order.size(), st);
  BatchRes* dres = ar.get<BatchRes>(count);
  ba.inst = dinst;
  ba.order = dorder;
  ba.res = dres;
  ba.count = (int32_t)order.size();
  ba.max_rounds = run.max_rounds;
  ba.literal = run.literal;
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  struct Ev2 {
    hipEvent_t a, b;
    ~Ev2() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};
  launch_batch_graph(ba, (int)slots, st, e0, e1);
  hres->assign(count, BatchRes{});
  d2h(hres->data(), dres, count, st);
  sync(st);
  float ms = 0.f;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  if (ws_bytes) *ws_bytes = (int64_t)ar.bytes_used();
  return ms;
}

int64_t heuristic_cells_cap(const mcc_problem* probs, const std::vector<int32_t>& ids) {
  int64_t n_max = 1;
  int32_t k_max = 1;
  for (int32_t i : ids) {
    n_max = std::max<int64_t>(n_max, probs[i].g.n);
    k_max = std::max<int32_t>(k_max, probs[i].k);
  }
  return std::min<int64_t>(std::max<int64_t>(n_max * k_max, (int64_t)1 << 18), kCellsCapMax);
}

}  // namespace

extern "C" {

int mcc_consensus_batch(const mcc_problem* probs, int32_t count, mcc_stats* stats,
                        mcc_batch_opts* opts) {
  if (count < 0 || (count > 0 && !probs)) return MCC_EINVAL;
  if (opts && opts->max_rounds < 0) return MCC_EINVAL;
  const int32_t max_rounds = opts && opts->max_rounds > 0 ? opts->max_rounds : 1000;
  const uint32_t flags = opts ? opts->flags : 0u;
  const int lanes = opts ? opts->lanes : 0;
  if (!batch_lanes_ok(lanes)) return MCC_EINVAL;
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  // launch shape: the caller's table, else the cache file, else built-in rules
  const mcc_tune_table* table = opts ? opts->tune : nullptr;
  mcc_tune_table loaded;
  if (!table && lanes == 0 && opts && opts->tune_cache_path &&
      mcc_tune_load(&loaded, opts->tune_cache_path) == MCC_OK)
    table = &loaded;
  int wgpc = opts && opts->wg_per_cu > 0 ? opts->wg_per_cu : (table ? table->wg_per_cu : 2);
  wgpc = std::max(1, std::min(wgpc, 8));
  std::vector<int32_t> status(count, MCC_OK);
  if (stats) memset(stats, 0, sizeof(mcc_stats) * (size_t)count);
  if (opts) {
    opts->solved_in_batch = 0;
    opts->ms_total = 0.f;
    opts->workspace_bytes = 0;
  }
  if (count == 0) return MCC_OK;

  // host-side argument checks, as mcc_consensus makes them
  std::vector<int32_t> eligible;
  std::vector<int32_t> fallback;
  VisibleRanges vis;
  for (int32_t i = 0; i < count; ++i) {
    if (!problem_ok(probs[i], true, vis)) {
      status[i] = MCC_EINVAL;
      continue;
    }
    if (probs[i].k > 256) fallback.push_back(i);
    else eligible.push_back(i);
  }

  int first_err = MCC_OK;
  try {
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    struct Ev2 {
      hipEvent_t a, b;
      ~Ev2() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } evg{e0, e1};
    HIPCK(hipEventRecord(e0, st));
    std::vector<BatchRes> hres(count);
    if (!eligible.empty()) {
      BatchRun run;
      run.probs = probs;
      run.ids = eligible;
      run.lanes.assign(count, 16);
      int64_t cells = 0;
      bool covered = table != nullptr;
      for (int32_t i : eligible) {
        const mcc_tune_entry* e = tune_lookup(table, probs[i].g.n, probs[i].k);
        if (!e) covered = false;
        else cells = std::max(cells, e->cells);
        run.lanes[i] = lanes ? lanes : (e ? e->lanes : default_lanes(probs[i].g.n));
      }
      run.cells_cap = covered ? std::min(kCellsCapMax, std::max(kCellsCapMin, pow2_ceil(cells)))
                              : heuristic_cells_cap(probs, eligible);
      run.wgpc = wgpc;
      run.max_rounds = max_rounds;
      run.literal = (flags & MCC_F_LITERAL) ? 1 : 0;
      int64_t ws = 0;
      run_batch(run, count, st, &hres, &ws);
      if (opts) opts->workspace_bytes = ws;
      for (int32_t i : eligible) {
        if (hres[i].status == kBatchTooBig) fallback.push_back(i);
        else if (hres[i].status == kBatchInvalid) status[i] = MCC_EINVAL;
        else if (opts) opts->solved_in_batch += 1;
      }
      for (int32_t i : eligible) {
        if (hres[i].status != 0 || !stats) continue;
        mcc_stats& o = stats[i];
        o.passes = hres[i].passes;
        o.converged = hres[i].converged;
        o.fallback_rounds = hres[i].fallback_rounds;
        o.clusters = hres[i].clusters;
        o.moves = hres[i].moves;
        o.candidate_evals = hres[i].candidate_evals;
        o.objective_init = hres[i].objective_init;
        o.objective = hres[i].objective;
        o.lanes_used = run.lanes[i];
      }
    }
    for (int32_t i : fallback) {
      const mcc_problem& p = probs[i];
      mcc_stats one;
      memset(&one, 0, sizeof one);
      one.max_rounds = max_rounds;
      one.flags = flags & MCC_F_LITERAL;
      one.stream = st;
      const int rc = mcc_consensus(&p.g, p.labels, p.k, p.init, p.out, &one);
      status[i] = rc;
      if (stats && rc == MCC_OK) stats[i] = one;
      if (opts) opts->workspace_bytes = std::max(opts->workspace_bytes, one.workspace_bytes);
    }
    HIPCK(hipEventRecord(e1, st));
    sync(st);
    if (opts) HIPCK(hipEventElapsedTime(&opts->ms_total, e0, e1));
  } catch (...) {
    return translate(std::current_exception());
  }
  for (int32_t i = 0; i < count; ++i) {
    if (status[i] != MCC_OK && first_err == MCC_OK) first_err = status[i];
    if (opts && opts->status) opts->status[i] = status[i];
  }
  return first_err;
}

int mcc_batch_tune(const mcc_problem* probs, int32_t count, const mcc_batch_opts* opts,
                   mcc_tune_table* table) {
  if (!table || count < 0 || (count > 0 && !probs)) return MCC_EINVAL;
  if (opts && (opts->max_rounds < 0 || !batch_lanes_ok(opts->lanes))) return MCC_EINVAL;
  memset(table, 0, sizeof *table);
  table->wg_per_cu = 2;
  std::vector<int32_t> ids;
  VisibleRanges vis;
  for (int32_t i = 0; i < count; ++i) {
    if (!problem_ok(probs[i], false, vis)) return MCC_EINVAL;
    if (probs[i].k <= 256 && probs[i].g.n > 0) ids.push_back(i);
  }
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  try {
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    int khz = 0;
    HIPCK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double ms_per_tick = khz > 0 ? 1.0 / khz : 0.0;
    // bucket of every instance
    std::vector<int32_t> bucket(count, -1);
    std::vector<std::pair<int, int>> keys;
    for (int32_t i : ids) {
      const std::pair<int, int> key{n_log2_of(probs[i].g.n), k_class_of(probs[i].k)};
      auto it = std::find(keys.begin(), keys.end(), key);
      if (it == keys.end()) {
        if ((int)keys.size() == MCC_TUNE_MAX_BUCKETS) return MCC_EINVAL;
        keys.push_back(key);
        it = keys.end() - 1;
      }
      bucket[i] = (int32_t)(it - keys.begin());
    }
    const int nb = (int)keys.size();
    table->count = nb;
    for (int j = 0; j < nb; ++j) {
      mcc_tune_entry& e = table->entry[j];
      e.n_log2 = keys[j].first;
      e.k_class = keys[j].second;
      e.lanes = 16;
      for (int c = 0; c < MCC_TUNE_LANES; ++c) e.ms[c] = -1.f;
    }
    if (ids.empty()) {
      if (opts && opts->tune_cache_path) return mcc_tune_save(table, opts->tune_cache_path);
      return MCC_OK;
    }
    Arena ar(st);
    // results go to scratch
    int64_t total_n = 0;
    for (int32_t i : ids) total_n += probs[i].g.n;
    int32_t* scratch = ar.get<int32_t>(total_n);
    BatchRun run;
    run.probs = probs;
    run.ids = ids;
    run.outs.assign(count, nullptr);
    int64_t off = 0;
    for (int32_t i : ids) {
      run.outs[i] = scratch + off;
      off += probs[i].g.n;
    }
    run.max_rounds = opts && opts->max_rounds > 0 ? opts->max_rounds : 1000;
    run.literal = opts && (opts->flags & MCC_F_LITERAL) ? 1 : 0;
    run.wgpc = opts && opts->wg_per_cu > 0 ? std::min(opts->wg_per_cu, 8) : 2;
    run.cells_cap = heuristic_cells_cap(probs, ids);  // larger tables still report their size
    std::vector<BatchRes> hres;
    std::vector<std::vector<double>> ms(nb, std::vector<double>(MCC_TUNE_LANES, 0.0));
    std::vector<int32_t> inst(nb, 0);
    std::vector<int64_t> cells(nb, 0);
    for (int c = 0; c < MCC_TUNE_LANES; ++c) {
      run.lanes.assign(count, kTuneLanes[c]);
      run_batch(run, count, st, &hres);
      for (int32_t i : ids) {
        const BatchRes& r = hres[i];
        const int j = bucket[i];
        cells[j] = std::max(cells[j], r.cells);
        if (r.status != 0) continue;
        ms[j][c] += (double)r.ticks * ms_per_tick;
        if (c == 0) inst[j] += 1;
      }
    }
    for (int j = 0; j < nb; ++j) {
      mcc_tune_entry& e = table->entry[j];
      e.instances = inst[j];
      e.cells = cells[j];
      int best = 2;
      for (int c = 0; c < MCC_TUNE_LANES; ++c) {
        e.ms[c] = inst[j] ? (float)ms[j][c] : -1.f;
        if (inst[j] && ms[j][c] < ms[j][best]) best = c;
      }
      e.lanes = kTuneLanes[best];
    }
    // resident workgroups per compute unit, with the chosen lanes and table size
    for (int32_t i : ids) run.lanes[i] = table->entry[bucket[i]].lanes;
    int64_t cmax = 0;
    for (int j = 0; j < nb; ++j) cmax = std::max(cmax, cells[j]);
    run.cells_cap = std::min(kCellsCapMax, std::max(kCellsCapMin, pow2_ceil(cmax)));
    // (only values whose workgroups take two or more instances each on
    // average: fewer problems than that say nothing about the full workload)
    std::vector<int> wgs;
    for (int wg : {1, 2, 4, 8})
      if ((int64_t)device_sms() * wg * 2 <= (int64_t)ids.size()) wgs.push_back(wg);
    if (wgs.size() < 2) wgs.clear();
    float best_ms = -1.f;
    for (int wg : wgs) {
      run.wgpc = wg;
      const float t = run_batch(run, count, st, &hres);
      if (best_ms < 0.f || t < best_ms) {
        best_ms = t;
        table->wg_per_cu = wg;
      }
    }
  } catch (...) {
    return translate(std::current_exception());
  }
  if (opts && opts->tune_cache_path) return mcc_tune_save(table, opts->tune_cache_path);
  return MCC_OK;
}

// ---------------------------------------------------------------------------
// Partition comparison and grouping of homogeneous partitions.
// ---------------------------------------------------------------------------
int mcc_compare(const int32_t* a, const int32_t* b, int64_t n, mcc_comparison* r, void* stream) {
  if (!r || n < 0 || n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  memset(r, 0, sizeof *r);
  if (n == 0) return MCC_OK;
  if (!device_visible(a) || !device_visible(b)) return MCC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    Arena ar(st);
    // the table of (cluster of a, label of b): dense ids of a as the
    // consensus, b as the one partition
    std::vector<const int32_t*> pa{a};
    Compacted ca;
    int32_t* err = ar.get<int32_t>(1);
    launch_fill_i32(err, 1, 0, st);
    int32_t herr = 0;
    std::vector<int32_t> maxlab;
    compact_labels(ar, pa, n, &ca, err, st, &herr, &maxlab);
    sync(st);
    if (herr & kErrNegLabel) return MCC_EINVAL;
    compact_labels_finish(ar, n, 1, maxlab, &ca, st);
    int32_t* da = ar.get<int32_t>(n);
    launch_dense_map(a, n, ca.scan, da, st);
    std::vector<const int32_t*> pb{b};
    Solve S;
    build_solve(ar, pb, n, da, false, nullptr, &S, st);
    const int32_t K0 = S.K0, Lb = S.lab.Lh[0];
    int32_t* rowmax = ar.get<int32_t>(K0);
    int32_t* colmax = ar.get<int32_t>(Lb);
    int32_t* colsum = ar.get<int32_t>(Lb);
    launch_fill_i32(rowmax, K0, 0, st);
    launch_fill_i32(colmax, Lb, 0, st);
    launch_fill_i32(colsum, Lb, 0, st);
    const int nb0 = cell_stats_blocks(S.total), nb1 = xlogx_blocks(K0), nb2 = xlogx_blocks(Lb);
    double* partial = ar.get<double>((int64_t)nb0 + nb1 + nb2);
    double* sums = ar.get<double>(3);
    int64_t* maxsum = ar.get<int64_t>(2);
    launch_fill_u64(reinterpret_cast<uint64_t*>(maxsum), 2, 0ull, st);
    launch_cell_stats(S.t, S.total, Lb, rowmax, colmax, colsum, partial, st);
    launch_xlogx(S.s, K0, partial + nb0, st);
    launch_xlogx(colsum, Lb, partial + nb0 + nb1, st);
    launch_sum_partials(partial, nb0, sums, st);
    launch_sum_partials(partial + nb0, nb1, sums + 1, st);
    launch_sum_partials(partial + nb0 + nb1, nb2, sums + 2, st);
    launch_sum_i32(rowmax, K0, maxsum, st);
    launch_sum_i32(colmax, Lb, maxsum + 1, st);
    int64_t acc[3], ms[2];
    double hs[3];
    d2h(acc, S.acc, 3, st);
    d2h(ms, maxsum, 2, st);
    d2h(hs, sums, 3, st);
    sync(st);
    r->mirkin = acc[0] + acc[1] - 2 * acc[2];
    r->split_join_ab = n - ms[0];
    r->split_join_ba = n - ms[1];
    r->split_join = r->split_join_ab + r->split_join_ba;
    r->vi = (hs[1] + hs[2] - 2.0 * hs[0]) / (double)n;
    r->rand = n > 1 ? (double)r->mirkin / ((double)n * (double)(n - 1)) : 0.0;
    r->clusters_a = K0;
    r->clusters_b = Lb;
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

int mcc_split_join_matrix(const int32_t* const* labels, int32_t k, int64_t n, int64_t* dist,
                          void* stream) {
  if (!dist || !labels || k < 1 || n < 0 || (int64_t)k * n >= ((int64_t)1 << 31))
    return MCC_EINVAL;
  memset(dist, 0, sizeof(int64_t) * (size_t)k * (size_t)k);
  if (n == 0 || k == 1) return labels_ok(labels, k) ? MCC_OK : MCC_EINVAL;
  if (!labels_ok(labels, k)) return MCC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  try {
    Arena ar(st);
    std::vector<const int32_t*> hptrs(labels, labels + k);
    Compacted lab;
    int32_t* err = ar.get<int32_t>(1);
    launch_fill_i32(err, 1, 0, st);
    int32_t herr = 0;
    std::vector<int32_t> maxlab;
    compact_labels(ar, hptrs, n, &lab, err, st, &herr, &maxlab);
    sync(st);
    if (herr & kErrNegLabel) return MCC_EINVAL;
    compact_labels_finish(ar, n, k, maxlab, &lab, st);
    std::vector<int32_t> Lh(k);
    d2h(Lh.data(), lab.L, k, st);
    // partition-major dense label ids
    int32_t* D = ar.get<int32_t>((int64_t)k * n);
    int64_t lo = 0;
    for (int i = 0; i < k; ++i) {
      launch_dense_map(hptrs[i], n, lab.scan + lo, D + (int64_t)i * n, st);
      lo += (int64_t)maxlab[i] + 1;
    }
    sync(st);
    // pairs in batches whose tables fit the cell budget; a pair too large
    // for it alone goes through mcc_compare (hashed tables)
    constexpr int64_t kPairCells = (int64_t)1 << 28;
    std::vector<int32_t> pi, pj;
    std::vector<int64_t> poff;
    auto flush = [&]() {
      if (pi.empty()) return;
      const int32_t np = (int32_t)pi.size();
      const int64_t cells = poff.back();
      Arena bar(st);
      int32_t* dpi = bar.get<int32_t>(np);
      int32_t* dpj = bar.get<int32_t>(np);
      int64_t* dpoff = bar.get<int64_t>(np + 1);
      h2d(dpi, bar.host(pi), np, st);
      h2d(dpj, bar.host(pj), np, st);
      h2d(dpoff, bar.host(poff), np + 1, st);
      int32_t* T = bar.get<int32_t>(cells);
      launch_fill_i32(T, cells, 0, st);
      int64_t* dd = bar.get<int64_t>(np);
      launch_pair_tables(D, n, dpi, dpj, dpoff, lab.L, np, T, st);
      launch_pair_split_join(T, dpi, dpj, dpoff, lab.L, np, n, dd, st);
      std::vector<int64_t> hd(np);
      d2h(hd.data(), dd, np, st);
      sync(st);
      for (int32_t p = 0; p < np; ++p) {
        dist[(int64_t)pi[p] * k + pj[p]] = hd[p];
        dist[(int64_t)pj[p] * k + pi[p]] = hd[p];
      }
      pi.clear();
      pj.clear();
      poff.clear();
    };
    for (int32_t i = 0; i < k; ++i)
      for (int32_t j = i + 1; j < k; ++j) {
        const int64_t cells = (int64_t)Lh[i] * Lh[j];
        if (cells > kPairCells) {
          mcc_comparison r;
          const int rc = mcc_compare(hptrs[i], hptrs[j], n, &r, stream);
          if (rc != MCC_OK) return rc;
          dist[(int64_t)i * k + j] = dist[(int64_t)j * k + i] = r.split_join;
          continue;
        }
        if (poff.empty()) poff.push_back(0);
        if (poff.back() + cells > kPairCells || (int64_t)pi.size() >= (1 << 20)) {
          flush();
          poff.push_back(0);
        }
        pi.push_back(i);
        pj.push_back(j);
        poff.push_back(poff.back() + cells);
      }
    flush();
    return MCC_OK;
  } catch (...) {
    return translate(std::current_exception());
  }
}

}  // extern "C"

namespace {

// Union-find over the k partitions.
struct Dsu {
  std::vector<int32_t> up;
  int32_t sets;
  explicit Dsu(int32_t k) : up(k), sets(k) {
    for (int32_t i = 0; i < k; ++i) up[i] = i;
  }
  int32_t find(int32_t x) {
    while (up[x] != x) x = up[x] = up[up[x]];
    return x;
  }
  void join(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (a < b) std::swap(a, b);
    up[a] = b;
    --sets;
  }
};

}  // namespace

extern "C" {

int mcc_group_from_distances(const int64_t* dist, int32_t k, int64_t lambda, int32_t* group,
                             int32_t* ngroups, int64_t* lambda_used) {
  if (!dist || !group || !ngroups || k < 1) return MCC_EINVAL;
  // edges in increasing distance; the number of groups after each distinct
  // distance comes from merging them in that order
  struct Edge {
    int64_t w;
    int32_t a, b;
  };
  std::vector<Edge> edges;
  edges.reserve((size_t)k * (k - 1) / 2);
  for (int32_t i = 0; i < k; ++i)
    for (int32_t j = i + 1; j < k; ++j) {
      if (dist[(int64_t)i * k + j] != dist[(int64_t)j * k + i] || dist[(int64_t)i * k + j] < 0)
        return MCC_EINVAL;
      edges.push_back({dist[(int64_t)i * k + j], i, j});
    }
  std::sort(edges.begin(), edges.end(), [](const Edge& x, const Edge& y) { return x.w < y.w; });
  int64_t lam = lambda;
  if (lam < 0) {
    // elbow: the distinct distance farthest below the chord of the curve
    // (distance, groups), both axes scaled to [0, 1]
    std::vector<int64_t> t;
    std::vector<int32_t> g;
    Dsu d(k);
    for (size_t e = 0; e < edges.size();) {
      const int64_t w = edges[e].w;
      for (; e < edges.size() && edges[e].w == w; ++e) d.join(edges[e].a, edges[e].b);
      t.push_back(w);
      g.push_back(d.sets);
    }
    lam = t.empty() ? 0 : t[0];
    const size_t m = t.size();
    if (m >= 3 && g[0] != g[m - 1]) {
      double best = 0.0;
      for (size_t j = 0; j < m; ++j) {
        const double x = (double)(t[j] - t[0]) / (double)(t[m - 1] - t[0]);
        const double y = ((double)g[j] - (double)g[m - 1]) / ((double)g[0] - (double)g[m - 1]);
        const double below = 1.0 - x - y;
        if (below > best) {
          best = below;
          lam = t[j];
        }
      }
    }
  }
  Dsu d(k);
  for (const Edge& e : edges) {
    if (e.w > lam) break;
    d.join(e.a, e.b);
  }
  std::vector<int32_t> id(k, -1);
  int32_t ng = 0;
  for (int32_t i = 0; i < k; ++i) {
    const int32_t root = d.find(i);
    if (id[root] < 0) id[root] = ng++;
    group[i] = id[root];
  }
  *ngroups = ng;
  if (lambda_used) *lambda_used = lam;
  return MCC_OK;
}

int mcc_group_partitions(const int32_t* const* labels, int32_t k, int64_t n, int64_t lambda,
                         int32_t* group, int32_t* ngroups, int64_t* lambda_used, int64_t* dist,
                         void* stream) {
  if (!group || !ngroups || k < 1) return MCC_EINVAL;
  std::vector<int64_t> own;
  int64_t* d = dist;
  if (!d) {
    own.assign((size_t)k * k, 0);
    d = own.data();
  }
  const int rc = mcc_split_join_matrix(labels, k, n, d, stream);
  if (rc != MCC_OK) return rc;
  return mcc_group_from_distances(d, k, lambda, group, ngroups, lambda_used);
}

int mcc_release_workspace(void) {
  {
    GraphCache& g = graph_cache();
    std::lock_guard<std::mutex> lock(g.m);
    for (auto& kv : g.g) destroy_graph(kv.second);
    g.g.clear();
  }
  ChunkCache& c = chunk_cache();
  std::lock_guard<std::mutex> lock(c.m);
  int cur = 0;
  (void)hipGetDevice(&cur);
  int rc = MCC_OK;
  for (auto& kv : c.free) {
    if (hipSetDevice(kv.first) != hipSuccess) rc = MCC_EDEVICE;
    for (const Chunk& k : kv.second)
      if (hipFree(k.p) != hipSuccess) rc = MCC_EDEVICE;
  }
  c.free.clear();
  c.bytes = 0;
  (void)hipSetDevice(cur);
  return rc;
}

int mcc_workspace_held(int64_t* bytes) {
  if (!bytes) return MCC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MCC_EDEVICE;
  ChunkCache& c = chunk_cache();
  std::lock_guard<std::mutex> lock(c.m);
  int64_t b = 0;
  auto it = c.free.find(dev);
  if (it != c.free.end())
    for (const Chunk& k : it->second) b += (int64_t)k.size;
  *bytes = b;
  return MCC_OK;
}

int mcc_workspace_bound(int64_t n, int64_t nnz, int32_t k, int64_t max_label, int64_t clusters,
                        uint32_t flags, int64_t* bytes) {
  if (!bytes || n < 0 || nnz < 0 || k < 1 || max_label < 0) return MCC_EINVAL;
  if ((int64_t)k * n >= ((int64_t)1 << 31)) return MCC_EINVAL;
  const int64_t nk = n * (int64_t)k;
  const int64_t span = std::min<int64_t>((int64_t)k * (max_label + 1), kMaxLabelFlags);
  const int64_t K0 = clusters > 0 ? std::min(clusters, n) : n;
  const int64_t sumL = std::min<int64_t>(span, nk);
  constexpr int64_t kChunk = (int64_t)16 << 20;
  // requests below a chunk are carved from chunks (at most as much again is
  // lost at chunk ends), larger ones get chunks of their own
  int64_t small = 0, big = 0;
  auto add = [&](int64_t b) {
    b = arena_round(b);
    if (b < kChunk) small += b;
    else big += b;
  };
  // labels and clusters: flags, scans, maps, row pointers
  add(4); add(8 * k); add(4 * k); add(8 * (k + 1));
  for (int j = 0; j < 3; ++j) add(4 * (span + 1));
  add(4 * (scan_tmp_elems(span) + 1)); add(4 * k);
  add(4 * (n + 1)); add(4 * (n + 1)); add(4 * (scan_tmp_elems(n) + 1));
  add(4 * n); add(4 * K0); add(4 * K0);
  // tables: the dense layouts (blocked, alignment, interleaved) when they
  // can be chosen, the hashed table when it can
  const int64_t dense_cap = dense_cells_max(n, k, K0, sumL, true);
  const int64_t dense_ub = K0 * sumL;  // clusters x labels, at most
  const bool can_hash = (flags & MCC_F_HASH_TABLES) ||
                        dense_ub > std::min<int64_t>(kMaxTableEntries, dense_cap);
  const int64_t dense = std::min<int64_t>(dense_ub, std::min<int64_t>(kMaxTableEntries, dense_cap));
  int64_t dsmall = 0, dbig = 0, hsmall = 0, hbig = 0;
  {
    std::swap(small, dsmall);
    std::swap(big, dbig);
    add(8 * (k + 1)); add(4 * dense);
    add(8 * (k + 1)); add(4 * ((int64_t)k * K0 + sumL));  // label sizes
    if (K0 <= kAlignMaxClusters) {
      add(8 * k * K0);
      for (int j = 0; j < 3; ++j) add(4 * (sumL + 1));
      add(8 * sumL); add(4 * sumL); add(4 * (scan_tmp_elems(sumL) + 1)); add(4 * k);
      add(4 * std::min<int64_t>(kMaxTableEntries, 2 * dense + (1 << 20)));
    }
    std::swap(small, dsmall);
    std::swap(big, dbig);
  }
  if (can_hash) {
    std::swap(small, hsmall);
    std::swap(big, hbig);
    int bits = 12;
    while (((int64_t)1 << bits) < 4 * nk) ++bits;
    add(8 * (k + 1)); add(16 * ((int64_t)1 << bits)); add(8); add(4 * sumL);
    add(4 * (K0 + 1)); add(4 * K0); add(4 * n); add(4 * (scan_tmp_elems(K0) + 1));
    // alignment to partition 0 for the row layout (its table is at most the
    // key table unless forced) and its label ids (at most L0 + L_i a partition)
    const int64_t L0 = std::min<int64_t>(max_label + 1, kAlignMaxClusters);
    if (L0 * sumL <= kRowsAlignCells) {
      add(4 * n); add(8 * (k + 1)); add(8 * (k + 1)); add(4 * L0 * sumL); add(8 * k * L0);
      add(4 * sumL); add(8 * sumL); add(4 * (sumL + 1)); add(4 * (sumL + 1));
      add(4 * (scan_tmp_elems(sumL) + 1)); add(4 * sumL); add(4 * k); add(n); add(8);
      add(8 * (k + 1)); add(4 * (sumL + k * L0));
      if (flags & MCC_F_HASH_ROWS) {
        int rbits = 12;
        while (((int64_t)1 << rbits) <= 2 * nk && ((int64_t)2 << rbits) * k < ((int64_t)1 << 31))
          ++rbits;
        add(8 * ((int64_t)1 << rbits)); add(4 * k * ((int64_t)1 << rbits));
      }
    }
    std::swap(small, hsmall);
    std::swap(big, hbig);
  }
  if (2 * hsmall + hbig > 2 * dsmall + dbig) {
    small += hsmall;
    big += hbig;
  } else {
    small += dsmall;
    big += dbig;
  }
  add(4 * nk); add(24);  // label rows, objective sums
  // per-pass state
  add(sizeof(Ctl)); add(8 * K0); add(4 * n); add(8 * n); add(4 * n); add(4 * n);
  add(8 * kPassCounters * kCounterStride); add(2 * n); add(4); add(4);
  if (flags & MCC_F_TRACE) add(8 * 4 * 1000);
  if (flags & MCC_F_ARC_CACHE) {
    add(4 * (n + 1)); add(4 * (n + 1)); add(4 * (scan_tmp_elems(n) + 1));
    add(4 * nnz); add(4 * nnz);
  }
  if (flags & MCC_F_SYMMETRIC) {
    for (int j = 0; j < 5; ++j) add(4 * n);
    add(4 * n * kCacheCand); add(8 * K0); add(4);
  }
  *bytes = big + 2 * small + kChunk;
  return MCC_OK;
}

int mcc_batch_workspace_bytes(const mcc_problem* probs, int32_t count,
                              const mcc_batch_opts* opts, int64_t* bytes) {
  if (!bytes || count < 0 || (count > 0 && !probs)) return MCC_EINVAL;
  *bytes = 0;
  const int lanes = opts ? opts->lanes : 0;
  if (!batch_lanes_ok(lanes)) return MCC_EINVAL;
  const mcc_tune_table* table = opts ? opts->tune : nullptr;
  mcc_tune_table loaded;
  if (!table && lanes == 0 && opts && opts->tune_cache_path &&
      mcc_tune_load(&loaded, opts->tune_cache_path) == MCC_OK)
    table = &loaded;
  int wgpc = opts && opts->wg_per_cu > 0 ? opts->wg_per_cu : (table ? table->wg_per_cu : 2);
  wgpc = std::max(1, std::min(wgpc, 8));
  std::vector<int32_t> eligible;
  int64_t single = 0;  // the largest bound of an instance solved by mcc_consensus
  for (int32_t i = 0; i < count; ++i) {
    const mcc_problem& p = probs[i];
    if (p.k < 1 || p.g.n < 0 || (int64_t)p.k * p.g.n >= ((int64_t)1 << 31)) return MCC_EINVAL;
    int64_t bound = 0;
    const int rc = mcc_workspace_bound(p.g.n, p.g.nnz, p.k, std::max<int64_t>(0, p.g.n - 1),
                                       0, 0, &bound);
    if (rc) return rc;
    if (p.k > 256) single = std::max(single, bound);
    else eligible.push_back(i);
  }
  if (!eligible.empty()) {
    int64_t cells = 0;
    bool covered = table != nullptr;
    for (int32_t i : eligible) {
      const mcc_tune_entry* e = tune_lookup(table, probs[i].g.n, probs[i].k);
      if (!e) covered = false;
      else cells = std::max(cells, e->cells);
    }
    const int64_t cap = covered ? std::min(kCellsCapMax, std::max(kCellsCapMin, pow2_ceil(cells)))
                                : heuristic_cells_cap(probs, eligible);
    const BatchSizes z = batch_sizes(probs, eligible, count, cap, wgpc);
    // carved from 16 MiB chunks (larger requests get their own)
    *bytes = 2 * z.bytes + ((int64_t)16 << 20);
  }
  *bytes = std::max(*bytes, single);
  return MCC_OK;
}

int mcc_tune_save(const mcc_tune_table* t, const char* path) {
  if (!t || !path || t->count < 0 || t->count > MCC_TUNE_MAX_BUCKETS) return MCC_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return MCC_EDEVICE;
  bool ok = fprintf(f, "mcc-tune 1\nwg_per_cu %d\nbuckets %d\n", t->wg_per_cu, t->count) > 0;
  for (int j = 0; j < t->count && ok; ++j) {
    const mcc_tune_entry& e = t->entry[j];
    ok = fprintf(f, "%d %d %d %d %lld", e.n_log2, e.k_class, e.lanes, e.instances,
                 (long long)e.cells) > 0;
    for (int c = 0; c < MCC_TUNE_LANES && ok; ++c) ok = fprintf(f, " %.6g", e.ms[c]) > 0;
    ok = ok && fputc('\n', f) != EOF;
  }
  if (fclose(f) != 0) ok = false;
  return ok ? MCC_OK : MCC_EDEVICE;
}

int mcc_tune_load(mcc_tune_table* t, const char* path) {
  if (!t || !path) return MCC_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return MCC_EINVAL;
  memset(t, 0, sizeof *t);
  int version = 0, wg = 0, count = 0;
  bool ok = fscanf(f, "mcc-tune %d wg_per_cu %d buckets %d", &version, &wg, &count) == 3 &&
            version == 1 && wg >= 1 && wg <= 8 && count >= 0 && count <= MCC_TUNE_MAX_BUCKETS;
  for (int j = 0; j < count && ok; ++j) {
    mcc_tune_entry& e = t->entry[j];
    long long cells = 0;
    ok = fscanf(f, "%d %d %d %d %lld", &e.n_log2, &e.k_class, &e.lanes, &e.instances, &cells) == 5;
    for (int c = 0; c < MCC_TUNE_LANES && ok; ++c) ok = fscanf(f, "%f", &e.ms[c]) == 1;
    e.cells = cells;
    ok = ok && e.n_log2 >= 0 && e.n_log2 <= 31 && e.k_class >= 0 && e.k_class <= 4 &&
         batch_lanes_ok(e.lanes) && e.lanes != 0 && e.cells >= 0 && e.instances >= 0;
  }
  fclose(f);
  if (!ok) {
    memset(t, 0, sizeof *t);
    return MCC_EINVAL;
  }
  t->count = count;
  t->wg_per_cu = wg;
  return MCC_OK;
}

}  // extern "C"
