// Host-side bounds checks made before a launch whose kernels write into a
// buffer sized elsewhere (plain C++, no HIP: also compiled by the CPU tests).
#pragma once

#include <cstdint>

namespace lsamg {

// A loop split over `split` ranges writes split x rows x width partial sums
// (width = right-hand sides of the launch) into `part`, which holds `cap`
// scalars.  True when the launch stays inside the buffer; a launch without a
// split (split <= 1) writes no partials.  Overflow-free for any inputs.
inline bool split_fits(int64_t split, int64_t rows, int64_t width, const void* part,
                       int64_t cap) {
  if (split <= 1) return true;
  if (part == nullptr || rows < 0 || width <= 0 || cap <= 0) return false;
  if (rows == 0) return true;
  const int64_t per = cap / width;         // rows x split that fit
  return split <= per / rows;
}

}  // namespace lsamg
