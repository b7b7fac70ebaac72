// Pass kernels instantiated for double elements.
#include "fft_passes.inc"

namespace tf {
template hipError_t launch_x_forward<double>(const double*, void*, const void*, int, int, int, RowMap, Batch, hipStream_t);
template hipError_t launch_x_inverse<double>(const void*, double*, const void*, int, int, int, RowMap, Batch, hipStream_t);
template hipError_t launch_y_pass<double>(void*, const void*, int, int, int, int, RowMap, int, Batch, hipStream_t);
template hipError_t launch_z_pass<double>(void*, const void*, const StepParams&, RowMap, int, double*, void*, int*, bool,
                                       Batch, hipStream_t);
template int z_diag_blocks<double>(int, int, int);
template hipError_t launch_z_current<double>(void*, const void*, const void*, const StepParams&, RowMap, hipStream_t);
template bool z_current_supported<double>(int);
}  // namespace tf
