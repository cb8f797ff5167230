// Reconstruction with intermediates in the library's fixed scratch array (see
// noalloc_ops.hip): the plan (mode order, largest intermediate) and the launcher.
#pragma once
#include <hip/hip_runtime.h>
#include "tdb_common.h"

// Doubles in the scratch array of each GPU (64 MiB): two halves for the ping-pong of
// the n-mode product chain.
#define NOALLOC_SCRATCH_DOUBLES (8ll * 1024 * 1024)

namespace tdb {

struct NoallocPlan {
  int p;
  int order[TDB_P];
  long long max_inter;   // largest intermediate (doubles); must fit half the scratch
};

NoallocPlan noalloc_plan(int p, const long long* dims, const int* ranks);
hipError_t noalloc_reconstruct(const NoallocPlan& pl, const long long* dims, const int* ranks, const double* C,
                               const double* const* U, int out_f32, void* out, hipStream_t s);

}  // namespace tdb
