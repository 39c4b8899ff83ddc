// lbfd_kernels_f32.hip -- float instantiations of the fused step, read and
// init kernels (D2Q9/D3Q19 x species bound 0/4/9/16).
#include "lbfd_device.h"
#include "lbfd_kernels.inc"
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
hipError_t launch_island_f32(int dim, int nsm, const StepArgs<float>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return hipSuccess;
    case 4: return launch_island_t<4>(dim, a, grid, s);
    case 9: return launch_island_t<9>(dim, a, grid, s);
    default: return launch_island_t<16>(dim, a, grid, s);
    }
}
}  // namespace lbfd
