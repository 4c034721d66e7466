// Instantiations of the uneven-batch persistent kernel for both precisions.
#include "batch_launch.hpp"
#include "fft_batch.hpp"

namespace dsfft {

template <class E>
static size_t batch_lds_bytes_t() {
    return (size_t)batch_lds_elems() * sizeof(E);
}

size_t batch_lds_bytes(int dtype) {
    return dtype == 0 ? batch_lds_bytes_t<uint32_t>() : batch_lds_bytes_t<f2_t>();
}

const void* batch_kernel_func(int dtype) {
    return dtype == 0 ? (const void*)&fft_batch_kernel<uint32_t> : (const void*)&fft_batch_kernel<f2_t>;
}

hipError_t launch_batch_reset(unsigned* ctl, int n, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, s, ctl, n);
    return hipGetLastError();
}

hipError_t launch_batch(int dtype, const void* in, void* out, void* ws, const void* lt,
                        const void* items, const int64_t* offs, int nitems, unsigned* ctl,
                        int spin_limit, int grid, hipStream_t s) {
    if (dtype == 0) {
        hipLaunchKernelGGL(fft_batch_kernel<uint32_t>, dim3(grid), dim3(kBatchThreads),
                           batch_lds_bytes_t<uint32_t>(), s, (const uint32_t*)in, (uint32_t*)out,
                           (uint32_t*)ws, (const TwH*)lt, (const BatchItem*)items, offs, nitems, ctl,
                           spin_limit);
    } else {
        hipLaunchKernelGGL(fft_batch_kernel<f2_t>, dim3(grid), dim3(kBatchThreads),
                           batch_lds_bytes_t<f2_t>(), s, (const f2_t*)in, (f2_t*)out, (f2_t*)ws,
                           (const TwF*)lt, (const BatchItem*)items, offs, nitems, ctl, spin_limit);
    }
    return hipGetLastError();
}

}  // namespace dsfft
