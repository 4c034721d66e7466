// Host-visible launch helpers of the uneven-batch kernel (kernels_batch.hip)
// and the work-item layout shared with batch.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace dsfft {

// Work item of the uneven-batch kernel (fields described in fft_batch.hpp).
struct HostBatchItem {
    int32_t cfg, nunits, first, log_m, phase, slot, reserved0, reserved1;
    int64_t in_off, out_off;
};
static_assert(sizeof(HostBatchItem) == 48, "work item layout");

// Configuration ids (same order as BatchCfg in fft_batch.hpp).
enum HostBatchCfg {
    HB_N2 = 0, HB_N4, HB_N8, HB_N16, HB_N32, HB_N64, HB_N128, HB_N256, HB_N512, HB_N1024,
    HB_N2048, HB_N4096, HB_N8192,
    HB_N1024_B, HB_N4096_B,
    HB_ROWS128, HB_COLS256, HB_ROWS256, HB_COLS512, HB_ROWS512, HB_N16384,
    HB_COUNT
};

constexpr int kHostBatchThreads = 512;

// Binary16 transforms of 2^15 points (too large for the batch kernel's LDS)
// run in a kernel of their own over a list of transform offsets.
constexpr int kBigListLog = 15;
constexpr int kBigListThreads = 1024;

constexpr int kMaxSingleLog = 14;      // sizes up to 2^14 run as whole-transform items
extern const int kSmallCfg[kMaxSingleLog + 1];   // their configuration per log2 N (1..14)
int cfg_upw(int cfg);                  // units per workgroup of a configuration

// Work list for transforms of sizes n[t] at element offsets off[t] (batch.cpp):
// phase-0 items (column items, then single-unit items) come first, `phase0`
// of them, then the phase-1 row items.  With big_log > 0, transforms of
// 2^big_log points go to `big` (offsets for the list kernel) instead.
void build_work(const int64_t* n, const int64_t* off, int64_t count, const int* cfg_choice,
                int big_log, std::vector<HostBatchItem>& items, std::vector<int64_t>& offs,
                std::vector<int64_t>& big, int64_t& ws_elems, int64_t& phase0);
// big_log for a dtype: binary16 2^15 transforms use the list kernel.
inline int big_log_for(int dtype) { return dtype == 0 ? kBigListLog : 0; }
int batch_resident_grid(int dtype, int device, int* out);

size_t batch_lds_bytes(int dtype);
const void* batch_kernel_func(int dtype);
size_t batch_big_lds_bytes();
const void* batch_big_func();
hipError_t launch_batch_big(const void* in, void* out, const void* lt, const int64_t* offs,
                            int64_t count, hipStream_t s);

// Queue words per batch or serving slot: (head, workgroups done) for each of
// the two phases; zero when allocated, and left zero by every launch.
constexpr int kQueueWords = 4;
// One phase: items first .. first + nitems - 1, queue words q[0..1].
hipError_t launch_batch(int dtype, const void* in, void* out, void* ws, const void* lt,
                        const void* items, const int64_t* offs, int first, int nitems,
                        unsigned* q, int grid, hipStream_t s);
// Both phases of a work list (phase 0 on ctl[0..1], phase 1 on ctl[2..3]) on
// stream s.
hipError_t launch_batch_phases(int dtype, const void* in, void* out, void* ws, const void* lt,
                               const void* items, const int64_t* offs, int phase0, int nitems,
                               unsigned* ctl, int grid0, int grid1, hipStream_t s);

}  // namespace dsfft
