// Host emulation of the grid group of HIP's cooperative groups -- TEST INFRASTRUCTURE.
//
// this_grid().sync() is a barrier of every work-item of a cooperative launch
// (hipLaunchCooperativeKernel, whose workgroups the emulation runs on host threads of their own).
#pragma once

#include <hip/hip_runtime.h>

namespace cooperative_groups {

struct grid_group {
    void sync() const { ::hipemu::grid_sync(); }
};

inline grid_group this_grid() { return grid_group{}; }

}  // namespace cooperative_groups
