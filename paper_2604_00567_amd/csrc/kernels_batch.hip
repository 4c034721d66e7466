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

// The binary16 2^15-point list kernel: 1024 threads (32 elements each),
// radix 2^5 passes, one transform per workgroup.
#define DSFFT_BIG_KERNEL fft_list_kernel<uint32_t, kBigListLog, 5, 5, 5, 5>

size_t batch_big_lds_bytes() {
    return (size_t)PassPlan<kBigListLog, 5, 5, 5, 0>::region() * sizeof(uint32_t);
}

const void* batch_big_func() { return (const void*)&DSFFT_BIG_KERNEL; }

hipError_t launch_batch_big(const void* in, void* out, const void* lt, const int64_t* offs,
                            int64_t count, hipStream_t s) {
    static_assert(kBigListThreads == (1 << (kBigListLog - 5)), "list kernel geometry");
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(DSFFT_BIG_KERNEL, dim3((unsigned)count), dim3(kBigListThreads),
                       batch_big_lds_bytes(), s, (const uint32_t*)in, (uint32_t*)out, (const TwH*)lt,
                       offs, count);
    return hipGetLastError();
}

hipError_t launch_batch(int dtype, const void* in, void* out, void* ws, const void* lt,
                        const void* items, const int64_t* offs, int first, int nitems,
                        unsigned* q, int grid, hipStream_t s) {
    if (dtype == 0) {
        hipLaunchKernelGGL(fft_batch_kernel<uint32_t>, dim3(grid), dim3(kBatchThreads),
                           batch_lds_bytes_t<uint32_t>(), s, (const uint32_t*)in, (uint32_t*)out,
                           (uint32_t*)ws, (const TwH*)lt, (const BatchItem*)items, offs, first, nitems,
                           q);
    } else {
        hipLaunchKernelGGL(fft_batch_kernel<f2_t>, dim3(grid), dim3(kBatchThreads),
                           batch_lds_bytes_t<f2_t>(), s, (const f2_t*)in, (f2_t*)out, (f2_t*)ws,
                           (const TwF*)lt, (const BatchItem*)items, offs, first, nitems, q);
    }
    return hipGetLastError();
}

hipError_t launch_batch_phases(int dtype, const void* in, void* out, void* ws, const void* lt,
                               const void* items, const int64_t* offs, int phase0, int nitems,
                               unsigned* ctl, int grid0, int grid1, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (phase0 > 0)
        e = launch_batch(dtype, in, out, ws, lt, items, offs, 0, phase0, ctl, grid0, s);
    if (e == hipSuccess && nitems > phase0)
        e = launch_batch(dtype, in, out, ws, lt, items, offs, phase0, nitems - phase0, ctl + 2,
                         grid1, s);
    return e;
}

}  // namespace dsfft
