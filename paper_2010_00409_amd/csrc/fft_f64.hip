// Pass kernels instantiated for double elements.
#include "fft_passes.inc"

namespace tf {
template hipError_t launch_x_forward<double>(const double*, void*, const void*, int, int, int, hipStream_t);
template hipError_t launch_x_inverse<double>(const void*, double*, const void*, int, int, int, hipStream_t);
template hipError_t launch_y_pass<double>(void*, const void*, int, int, int, int, hipStream_t);
template hipError_t launch_z_pass<double>(void*, const void*, const StepParams&, int, double*, int*, hipStream_t);
template int z_pass_blocks<double>(int, int, int);
}  // namespace tf
