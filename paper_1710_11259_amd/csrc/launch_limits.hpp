// Launch-size limits shared by the host code (pure C++, no HIP types).
#pragma once

#include <cstdint>

namespace fps {

// A 1-D launch of `threads`-wide workgroups may hold at most this many
// workgroups: the grid's work-item count (workgroups x threads) must stay
// below 2^32.
constexpr int64_t max_workgroups_1d(int threads) {
  return (int64_t)0xFFFFFFFFu / (int64_t)threads;
}

// Whether `workgroups` workgroups of 256 threads fit one 1-D launch (the
// batched element-wise passes).
constexpr bool elem_launch_fits(int64_t workgroups) {
  return workgroups >= 0 && workgroups <= max_workgroups_1d(256);
}

}  // namespace fps
