// Internal declarations of the batched persistent solver (batch.hip).
#pragma once

#include "impl.h"

namespace mcc {

// One instance of a batch (device copy).
struct BatchInst {
  int64_t n, nnz;
  const int64_t* row_ptr;
  const int32_t* col;
  const int32_t* const* labels;  // device array of k device pointers
  const int32_t* init;           // null: singletons
  int32_t* out;
  int32_t k;
  int32_t lanes;  // lanes per vertex in the scorer: 4, 8, 16, 32 or 64
};

// Per-instance result written by the kernel.
struct BatchRes {
  int32_t status;  // 0, kBatchTooBig (solve elsewhere) or kBatchInvalid
  int32_t passes, converged, fallback_rounds, clusters;
  int32_t pad;
  int64_t moves, candidate_evals, objective_init, objective;
  int64_t cells;  // table cells the instance needs (0 if it failed earlier)
  int64_t ticks;  // device wall-clock ticks the workgroup spent on it
};

constexpr int32_t kBatchTooBig = 1;
constexpr int32_t kBatchInvalid = 2;

// Workspace: slot s of each array starts at base + s * (per-slot length).
struct BatchWs {
  int64_t n_max;      // vertices per slot
  int32_t k_max;      // partitions per slot
  int32_t pad;
  int64_t cells_cap;  // table cells per slot
  int64_t flag_cap;   // flag/scan entries per slot (label values, cluster ids)
  int32_t* C;
  int32_t* rawid;
  int32_t* prop;
  int64_t* dprop;
  int32_t* s;
  uint64_t* owner;
  int32_t* Lvm;
  int32_t* N;
  int32_t* flags;
};

struct BatchArgs {
  const BatchInst* inst;
  const int32_t* order;  // queue order (largest work first)
  BatchRes* res;
  // Queue position counter, never reset: the launch's positions start at
  // qbase, and every workgroup takes one position past the last instance
  // before it stops, so the next launch's base is qbase + count + grid.
  unsigned long long* queue;
  unsigned long long qbase;
  int32_t count;
  int32_t max_rounds;
  int32_t literal;
  int32_t pad;
  BatchWs ws;
};

bool batch_lanes_ok(int lanes);
void launch_batch(const BatchArgs& a, int grid, hipStream_t st);
// The persistent kernel, for a graph kernel node (one BatchArgs argument).
const void* batch_kernel();

}  // namespace mcc
