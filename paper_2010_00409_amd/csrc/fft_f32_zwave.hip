// The one-wave-per-mode z kernels of the shipped plans (z variant 11 at 512,
// variant 7 at 256), in a translation unit of its own: build.py compiles it
// with the memory-clause scheduling strategy, which groups the kernels'
// memory instructions (on MI355X the 512^3 z pass 1.331 -> 1.317 ms, the
// 256^3 one 0.172 -> 0.169 ms), while the other pass kernels keep the
// default strategy (under which the y passes run 0.5% faster).
// fft_f32.hip declares both instantiations extern.
#include "fft_passes.inc"

namespace tf {
template __global__ void k_z_wave<4, 1, false, 2>(float2* __restrict__, const float2* __restrict__, StepParams,
                                                  RowMap, Batch);
template __global__ void k_z_wave256<4, 3>(float2* __restrict__, const float2* __restrict__, StepParams, RowMap, Batch);
}  // namespace tf
