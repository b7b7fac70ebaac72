// The 512-point one-wave-per-mode z kernel of the shipped 512^3 plan (z
// variant 11), in a translation unit of its own: build.py compiles it with
// the memory-clause scheduling strategy, which groups the kernel's memory
// instructions (the z pass 1.339 -> 1.327 ms on MI355X), while the other
// pass kernels keep the default strategy (under which the y passes run
// 0.5% faster).  fft_f32.hip declares the instantiation extern.
#include "fft_passes.inc"

namespace tf {
template __global__ void k_z_wave<4, 1, false, 2>(float2* __restrict__, const float2* __restrict__, StepParams,
                                                  RowMap, Batch);
}  // namespace tf
