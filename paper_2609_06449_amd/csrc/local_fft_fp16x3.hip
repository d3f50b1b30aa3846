// LocalFFT kernels whose radix-16 butterflies run on MFMA in the FP16x3
// split form (stages.h); everything else as in the FP32 kernels.
#include "local_fft_kernels.h"

namespace paco {

const void *fast_kernel_fp16x3(int log2n, int mode, int tb, int groups)
{
    return fast_kernel_t<kPrecFP16x3>(log2n, mode, tb, groups);
}

const void *generic_kernel_fp16x3(int log2n, bool pre, bool gen)
{
    return generic_kernel_t<kPrecFP16x3>(log2n, pre, gen);
}

}  // namespace paco
