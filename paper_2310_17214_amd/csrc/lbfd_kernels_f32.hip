// lbfd_kernels_f32.hip -- float instantiations of the fused step, read and
// init kernels (D2Q9/D3Q19 x species bound 0/4/9/16), the FP64 reaction
// island and the chemistry surrogate kernels.
#include "lbfd_device.h"
#include "lbfd_kernels.inc"
#include "lbfd_mlp.inc"
#include "lbfd_launch.h"

namespace lbfd {
hipError_t launch_step_f32(int dim, int nsm, const StepArgs<float>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_step_t<float, 0>(dim, a, grid, s);
    case 4: return launch_step_t<float, 4>(dim, a, grid, s);
    case 9: return launch_step_t<float, 9>(dim, a, grid, s);
    default: return launch_step_t<float, 16>(dim, a, grid, s);
    }
}
hipError_t launch_p0_sum_f32(const float* T, const float* Y, int N, int ns, const Par<float>* P,
                              double* part, hipStream_t s) {
    return launch_p0_sum_t<float>(T, Y, N, ns, P, part, s);
}
hipError_t launch_macro_f32(int dim, int nsm, const MacroArgs<float>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_macro_t<float, 0>(dim, a, grid, s);
    case 4: return launch_macro_t<float, 4>(dim, a, grid, s);
    case 9: return launch_macro_t<float, 9>(dim, a, grid, s);
    default: return launch_macro_t<float, 16>(dim, a, grid, s);
    }
}
hipError_t launch_init_f32(int dim, int nsm, const InitArgs<float>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_init_t<float, 0>(dim, a, grid, s);
    case 4: return launch_init_t<float, 4>(dim, a, grid, s);
    case 9: return launch_init_t<float, 9>(dim, a, grid, s);
    default: return launch_init_t<float, 16>(dim, a, grid, s);
    }
}

int step_tile_h_f32(int dim, int nsm) {
    switch (nsm) {
    case 0: return tile_h_t<float, 0>(dim);
    case 4: return tile_h_t<float, 4>(dim);
    case 9: return tile_h_t<float, 9>(dim);
    default: return tile_h_t<float, 16>(dim);
    }
}
hipError_t launch_island_f32(int dim, int nsm, const StepArgs<float>& a, hipStream_t s) {
    switch (nsm) {
    case 0: return hipSuccess;
    case 4: return launch_island_t<4>(dim, a, s);
    case 9: return launch_island_t<9>(dim, a, s);
    default: return launch_island_t<16>(dim, a, s);
    }
}
hipError_t launch_mlp_step_f32(int dim, int nsm, const StepArgs<float>& a, const SurWeights* gw,
                               const SurPar* sp, int grid, hipStream_t s) {
    switch (nsm) {
    case 4: return launch_mlp_step_t<4>(dim, a, gw, sp, grid, s);
    case 9: return launch_mlp_step_t<9>(dim, a, gw, sp, grid, s);
    case 16: return launch_mlp_step_t<16>(dim, a, gw, sp, grid, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_mlp_eval_f32(int nsm, const float* T, const float* Y, int n, float* raw, float* w,
                               int* fb, const Par<float>* P, const SurWeights* gw,
                               const SurPar* sp, int grid, hipStream_t s) {
    switch (nsm) {
    case 4: return launch_mlp_eval_t<4>(T, Y, n, raw, w, fb, P, gw, sp, grid, s);
    case 9: return launch_mlp_eval_t<9>(T, Y, n, raw, w, fb, P, gw, sp, grid, s);
    case 16: return launch_mlp_eval_t<16>(T, Y, n, raw, w, fb, P, gw, sp, grid, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_sample_f32(int nsm, const float* T, const float* Y, int N, const int* cells,
                             int n, float* x, float* y, const Par<double>* PD, float p_in,
                             hipStream_t s) {
    switch (nsm) {
    case 4: return launch_sample_t<4>(T, Y, N, cells, n, x, y, PD, p_in, s);
    case 9: return launch_sample_t<9>(T, Y, N, cells, n, x, y, PD, p_in, s);
    case 16: return launch_sample_t<16>(T, Y, N, cells, n, x, y, PD, p_in, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_si_mask_f32(int dim, const uint8_t* solid, const Par<float>* P, uint32_t* mask,
                                int n, hipStream_t s) {
    return launch_si_mask_t<float>(dim, solid, P, mask, n, s);
}
hipError_t launch_halo_f32(const HaloArgs<float>& a, hipStream_t s) {
    return launch_halo_t<float>(a, s);
}
}  // namespace lbfd
