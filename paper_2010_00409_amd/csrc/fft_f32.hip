// Pass kernels instantiated for float elements.
#include "fft_passes.inc"

namespace tf {
// compiled in fft_f32_zwave.hip with its own scheduling strategy
extern template __global__ void k_z_wave<4, 1, false, 2>(float2* __restrict__, const float2* __restrict__, StepParams,
                                                         RowMap, Batch);
extern template __global__ void k_z_wave256<4, 3>(float2* __restrict__, const float2* __restrict__, StepParams, RowMap,
                                                  Batch);
template hipError_t launch_x_forward<float>(const float*, void*, const void*, int, int, int, RowMap, Batch, hipStream_t);
template hipError_t launch_x_inverse<float>(const void*, float*, const void*, int, int, int, RowMap, Batch, hipStream_t);
template hipError_t launch_y_pass<float>(void*, const void*, int, int, int, int, RowMap, int, Batch, hipStream_t);
template hipError_t launch_z_pass<float>(void*, const void*, const StepParams&, RowMap, int, double*, void*, int*, bool,
                                       Batch, hipStream_t);
template int z_diag_blocks<float>(int, int, int);
template hipError_t launch_z_current<float>(void*, const void*, const void*, const StepParams&, RowMap, hipStream_t);
template bool z_current_supported<float>(int);
}  // namespace tf

namespace tf {
bool fft_length_supported(int n) {
    switch (n) {
#define X(m) case m: return true;
        TF_FOR_LENGTHS(X)
#undef X
    }
    return false;
}
}  // namespace tf
