// lbfd_launch.h -- internal launch entry points of the per-precision kernel
// translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "lbfd_device.h"

namespace lbfd {
hipError_t launch_step_f32(int dim, int nsm, const StepArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_step_f64(int dim, int nsm, const StepArgs<double>& a, int grid, hipStream_t s);
hipError_t launch_macro_f32(int dim, int nsm, const MacroArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_macro_f64(int dim, int nsm, const MacroArgs<double>& a, int grid, hipStream_t s);
hipError_t launch_init_f32(int dim, int nsm, const InitArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_init_f64(int dim, int nsm, const InitArgs<double>& a, int grid, hipStream_t s);
hipError_t launch_island_f32(int dim, int nsm, const StepArgs<float>& a, int grid, hipStream_t s);
// cell rows per workgroup tile of the step kernel (tiles are 32 cells wide)
int step_tile_h_f32(int dim, int nsm);
int step_tile_h_f64(int dim, int nsm);
}  // namespace lbfd
