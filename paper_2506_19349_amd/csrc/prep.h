// Host side of the device graph: ownership of the device arrays and the
// preparation entry point.
#pragma once

#include <string>
#include <vector>

#include "engine.h"

namespace sssp {

struct GraphHost {
  int device = 0;
  DevGraph h{};              // host copy holding device pointers
  DevGraph* d = nullptr;     // device copy
  std::vector<void*> allocs;
  size_t bytes = 0;
  int32_t nonisolated = 0;
  int32_t distinct_degrees = 0;
  int32_t max_degree = 0;
};

// Returns 0 on success or a negative sssp_status; *msg explains failures.
int prep_graph(int32_t n, const int32_t* rowptr, const int32_t* colidx, const uint32_t* weight,
               int flags, GraphHost* out, std::string* msg);

void free_graph(GraphHost* g);

// Launch helpers exported by the engine translation unit.
hipError_t launch_high_d(const int32_t* deg_vals, const uint32_t* cnt, int32_t D, uint32_t* out_h,
                         unsigned long long* out_mass, hipStream_t stream);

}  // namespace sssp
