// CPU stand-in for <hip/hip_cooperative_groups.h> (see hip_runtime.h).
#pragma once
#include "hip_runtime.h"
namespace cooperative_groups {
struct grid_group {
    void sync() const { simt::grid_sync(); }
};
inline grid_group this_grid() { return grid_group{}; }
}  // namespace cooperative_groups
