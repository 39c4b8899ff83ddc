// lbfd_launch.h -- internal launch entry points of the per-precision kernel
// translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "lbfd_device.h"
#include "lbfd_mlp.h"

namespace lbfd {
hipError_t launch_step_f32(int dim, int nsm, const StepArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_step_f64(int dim, int nsm, const StepArgs<double>& a, int grid, hipStream_t s);
hipError_t launch_macro_f32(int dim, int nsm, const MacroArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_macro_f64(int dim, int nsm, const MacroArgs<double>& a, int grid, hipStream_t s);
hipError_t launch_init_f32(int dim, int nsm, const InitArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_init_f64(int dim, int nsm, const InitArgs<double>& a, int grid, hipStream_t s);
// FP32 mode: compaction of the flagged cells and their FP64 reaction step
hipError_t launch_island_f32(int dim, int nsm, const StepArgs<float>& a, hipStream_t s);
// chemistry surrogate (FP32 only; species buckets 4, 9, 16)
hipError_t launch_mlp_step_f32(int dim, int nsm, const StepArgs<float>& a, const SurWeights* gw,
                               const SurPar* sp, int grid, hipStream_t s);
hipError_t launch_mlp_eval_f32(int nsm, const float* T, const float* Y, int n, float* raw, float* w,
                               int* fb, const Par<float>* P, const SurWeights* gw,
                               const SurPar* sp, int grid, hipStream_t s);
hipError_t launch_sample_f32(int nsm, const float* T, const float* Y, int N, const int* cells,
                             int n, float* x, float* y, const Par<double>* PD, float p_in,
                             hipStream_t s);
// closed domain: per-workgroup sums of M / T (P0_PARTS partials)
hipError_t launch_p0_sum_f32(const float* T, const float* Y, int N, int ns, const Par<float>* P,
                             double* part, hipStream_t s);
hipError_t launch_p0_sum_f64(const double* T, const double* Y, int N, int ns,
                             const Par<double>* P, double* part, hipStream_t s);
// sharp-interface mode: link masks from the per-cell solid flags
hipError_t launch_si_mask_f32(int dim, const uint8_t* solid, const Par<float>* P, uint32_t* mask,
                              int n, hipStream_t s);
hipError_t launch_si_mask_f64(int dim, const uint8_t* solid, const Par<double>* P, uint32_t* mask,
                              int n, hipStream_t s);
// halo planes of an x face
hipError_t launch_halo_f32(const HaloArgs<float>& a, hipStream_t s);
hipError_t launch_halo_f64(const HaloArgs<double>& a, hipStream_t s);
// cell rows per workgroup tile of the step kernel (tiles are 64 cells wide)
int step_tile_h_f32(int dim, int nsm);
int step_tile_h_f64(int dim, int nsm);
}  // namespace lbfd
