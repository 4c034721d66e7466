// Instantiations of the uneven-batch persistent kernel for both precisions.
#include "batch_launch.hpp"
#include "fft_batch.hpp"

namespace dsfft {

template <class E>
static size_t batch_lds_bytes_t() {
    return batch_prefix_bytes<E>() + (size_t)batch_lds_elems() * sizeof(E);
}

static_assert(batch_prefix_bytes<uint32_t>() + (size_t)batch_lds_elems() * sizeof(uint32_t) <= kLdsBytes &&
                  batch_prefix_bytes<f2_t>() + (size_t)batch_lds_elems() * sizeof(f2_t) <= kLdsBytes,
              "the persistent kernel fits a workgroup's LDS");

size_t batch_lds_bytes(int dtype) {
    return dtype == 0 ? batch_lds_bytes_t<uint32_t>() : batch_lds_bytes_t<f2_t>();
}

const void* batch_kernel_func(int dtype) {
    return dtype == 0 ? (const void*)&fft_batch_kernel<uint32_t> : (const void*)&fft_batch_kernel<f2_t>;
}

// The binary16 list kernels, 1024 threads each: 2^16 points with 64 elements
// per lane (radix 2^6, 2^5, 2^5; each exchange in two rounds of half the rows)
// and 2^15 points with 32 (radix 2^5 passes); the middle pass reads table
// entries [L0, L0 R) from the LDS prefix (2048 and 1024 entries).
#define DSFFT_LIST16 fft_list_kernel<uint32_t, 16, 6, 6, 5, 5, 2048>
#define DSFFT_LIST15 fft_list_kernel<uint32_t, 15, 5, 5, 5, 5, 1024>
static_assert(kListLog[0] == 16 && kListLog[1] == 15 && kListThreads == (1 << (16 - 6)) &&
                  kListThreads == (1 << (15 - 5)),
              "list kernel geometry");

size_t batch_list_lds_bytes(int list) {
    return list == 0 ? 2048 * sizeof(TwH) +
                           unit_lds_elems<uint32_t, 6, MODE_SMALL, 1, PassPlan<16, 6, 5, 5, 0>>() * sizeof(uint32_t)
                     : 1024 * sizeof(TwH) +
                           unit_lds_elems<uint32_t, 5, MODE_SMALL, 1, PassPlan<15, 5, 5, 5, 0>>() * sizeof(uint32_t);
}
static_assert(2048 * sizeof(TwH) + unit_lds_elems<uint32_t, 6, MODE_SMALL, 1, PassPlan<16, 6, 5, 5, 0>>() *
                                       sizeof(uint32_t) <= kLdsBytes &&
                  1024 * sizeof(TwH) + unit_lds_elems<uint32_t, 5, MODE_SMALL, 1, PassPlan<15, 5, 5, 5, 0>>() *
                                           sizeof(uint32_t) <= kLdsBytes,
              "list kernels fit a workgroup's LDS");

const void* batch_list_func(int list) {
    return list == 0 ? (const void*)&DSFFT_LIST16 : (const void*)&DSFFT_LIST15;
}

hipError_t launch_batch_list(int list, const void* in, void* out, const void* lt, const int64_t* offs,
                             int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (count > 0x7fffffffLL || list < 0 || list >= kNumLists) return hipErrorInvalidValue;
    if (list == 0)
        hipLaunchKernelGGL(DSFFT_LIST16, dim3((unsigned)count), dim3(kListThreads), batch_list_lds_bytes(0), s,
                           (const uint32_t*)in, (uint32_t*)out, (const TwH*)lt, offs, count);
    else
        hipLaunchKernelGGL(DSFFT_LIST15, dim3((unsigned)count), dim3(kListThreads), batch_list_lds_bytes(1), s,
                           (const uint32_t*)in, (uint32_t*)out, (const TwH*)lt, offs, count);
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
