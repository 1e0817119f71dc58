// Capacities of the solver's work lists that follow from a bound rather than
// from the graph alone. Plain C++ (no HIP), so that the bound can be checked
// on its own.
#pragma once

#include <stdint.h>

namespace sssp {

// Entries of one heavy-chunk list. A tick emits, for every item whose edge
// range is longer than the split threshold h (h >= min_split), ceil(size /
// chunk) chunks of that range. The range lies in the item's row, and a vertex
// is an item of at most two segments of one tick (the pending list and the
// pull list of a step's first round; every other segment lists a vertex at
// most once, and the segments of one tick are either those of a first round
// or the frontier and the previous tick's chunks, which emit none). So the
// ranges of one tick sum to at most 2 nnz entries and number at most twice
// the rows longer than min_split, and
//   chunks < sum(size / chunk + 1) <= 2 nnz / chunk + 2 heavy_rows,
// heavy_rows = #{v : deg(v) > min_split}.
inline int64_t heavy_list_capacity(int64_t nnz, int64_t heavy_rows, int64_t chunk) {
  return 2 * ((nnz + chunk - 1) / chunk) + 2 * heavy_rows + 16;
}

}  // namespace sssp
