// lbfd_kernels_f64.hip -- double instantiations of the fused step, read and
// init kernels (D2Q9/D3Q19 x species bound 0/4/9/16).
#include "lbfd_device.h"
#include "lbfd_kernels.inc"
#include "lbfd_launch.h"

namespace lbfd {
hipError_t launch_step_f64(int dim, int nsm, const StepArgs<double>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_step_t<double, 0>(dim, a, grid, s);
    case 4: return launch_step_t<double, 4>(dim, a, grid, s);
    case 9: return launch_step_t<double, 9>(dim, a, grid, s);
    default: return launch_step_t<double, 16>(dim, a, grid, s);
    }
}
hipError_t launch_p0_sum_f64(const double* T, const double* Y, int N, int ns, const Par<double>* P,
                              double* part, hipStream_t s) {
    return launch_p0_sum_t<double>(T, Y, N, ns, P, part, s);
}
hipError_t launch_macro_f64(int dim, int nsm, const MacroArgs<double>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_macro_t<double, 0>(dim, a, grid, s);
    case 4: return launch_macro_t<double, 4>(dim, a, grid, s);
    case 9: return launch_macro_t<double, 9>(dim, a, grid, s);
    default: return launch_macro_t<double, 16>(dim, a, grid, s);
    }
}
hipError_t launch_init_f64(int dim, int nsm, const InitArgs<double>& a, int grid, hipStream_t s) {
    switch (nsm) {
    case 0: return launch_init_t<double, 0>(dim, a, grid, s);
    case 4: return launch_init_t<double, 4>(dim, a, grid, s);
    case 9: return launch_init_t<double, 9>(dim, a, grid, s);
    default: return launch_init_t<double, 16>(dim, a, grid, s);
    }
}

int step_tile_h_f64(int dim, int nsm) {
    switch (nsm) {
    case 0: return tile_h_t<double, 0>(dim);
    case 4: return tile_h_t<double, 4>(dim);
    case 9: return tile_h_t<double, 9>(dim);
    default: return tile_h_t<double, 16>(dim);
    }
}
hipError_t launch_si_mask_f64(int dim, const uint8_t* solid, const Par<double>* P, uint32_t* mask,
                                int n, hipStream_t s) {
    return launch_si_mask_t<double>(dim, solid, P, mask, n, s);
}
hipError_t launch_halo_f64(const HaloArgs<double>& a, hipStream_t s) {
    return launch_halo_t<double>(a, s);
}
}  // namespace lbfd
