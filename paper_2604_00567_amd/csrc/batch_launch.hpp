// Host-visible launch helpers of the uneven-batch kernel (kernels_batch.hip)
// and the work-item layout shared with batch.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace dsfft {

// Mirrors BatchItem in fft_batch.hpp (checked by a static_assert there).
struct HostBatchItem {
    int32_t cfg, nunits, first, log_m, wait_slot, wait_need, post_slot, reserved;
    int64_t in_off, out_off;
};

// Configuration ids (same order as BatchCfg in fft_batch.hpp).
enum HostBatchCfg {
    HB_N2 = 0, HB_N4, HB_N8, HB_N16, HB_N32, HB_N64, HB_N128, HB_N256, HB_N512, HB_N1024,
    HB_N2048, HB_N4096, HB_N8192,
    HB_N1024_B, HB_N4096_B,
    HB_COLS128, HB_ROWS128, HB_COLS256, HB_ROWS256, HB_COLS512, HB_ROWS512,
    HB_COUNT
};

constexpr int kHostBatchThreads = 256;
constexpr int kSpinLimit = 1 << 22;    // dependency-wait sleeps (~512 cycles each): about a second

extern const int kSmallCfg[14];        // single-unit configuration per log2 N (1..13)
int cfg_upw(int cfg);                  // units per workgroup of a configuration

// Work list for transforms of sizes n[t] at element offsets off[t] (batch.cpp).
void build_work(const int64_t* n, const int64_t* off, int64_t count, const int* cfg_choice,
                std::vector<HostBatchItem>& items, std::vector<int64_t>& offs, int64_t& ws_elems,
                int& nslots);
int batch_resident_grid(int dtype, int device, int* out);

size_t batch_lds_bytes(int dtype);
const void* batch_kernel_func(int dtype);
hipError_t launch_batch_reset(unsigned* ctl, int n, hipStream_t s);
hipError_t launch_batch(int dtype, const void* in, void* out, void* ws, const void* lt,
                        const void* items, const int64_t* offs, int nitems, unsigned* ctl,
                        int spin_limit, int grid, hipStream_t s);

}  // namespace dsfft
