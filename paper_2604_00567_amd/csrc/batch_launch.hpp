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
    HB_N128_B, HB_N256_B, HB_N512_B, HB_N2048_B,
    HB_COUNT
};

constexpr int kHostBatchThreads = 512;

constexpr int kMaxSingleLog = 14;      // sizes up to 2^14 run as whole-transform items

// Binary16 transforms of 2^16 and 2^15 points (too large for the batch
// kernel's LDS) run whole in list kernels of their own, one transform per
// 1024-thread workgroup, over lists of transform offsets: list 0 holds the
// 2^16-point transforms, list 1 the 2^15-point ones.
constexpr int kNumLists = 2;
constexpr int kListLog[kNumLists] = {16, 15};
constexpr int kListThreads = 1024;
// Lists a dtype uses (binary16 both, binary32 none) and the largest size it
// runs whole; larger transforms take the column/row split (and a workspace).
inline int lists_for(int dtype) { return dtype == 0 ? kNumLists : 0; }
inline int max_whole_log(int dtype) { return dtype == 0 ? kListLog[0] : kMaxSingleLog; }
extern const int kSmallCfg[kMaxSingleLog + 1];   // their configuration per log2 N (1..14)
// The alternative configuration per log2 N that the batch tuner weighs
// against kSmallCfg (another radix split, units per workgroup and elements per
// lane), -1 where there is none.
extern const int kAltCfg[kMaxSingleLog + 1];
int cfg_upw(int cfg);                  // units per workgroup of a configuration

// Work list for transforms of sizes n[t] at element offsets off[t] (batch.cpp):
// phase-0 items (column items, then single-unit items) come first, `phase0`
// of them, then the phase-1 row items.  With nlists > 0, transforms of
// 2^kListLog[i] points (i < nlists) go to the list kernels instead: `lists`
// holds list 0's offsets, then list 1's, nlist[i] of each.
void build_work(const int64_t* n, const int64_t* off, int64_t count, const int* cfg_choice,
                int nlists, std::vector<HostBatchItem>& items, std::vector<int64_t>& offs,
                std::vector<int64_t>& lists, int64_t* nlist, int64_t& ws_elems, int64_t& phase0);
// Work items that `count` transforms of 2^m points add to a work list built
// with kSmallCfg: whole transforms of one size share items of cfg_upw units,
// list-kernel sizes take none, and each split transform takes its column and
// row items.
int64_t work_items_of_class(int dtype, int m, int64_t count);
int batch_resident_grid(int dtype, int device, int* out);

size_t batch_lds_bytes(int dtype);
const void* batch_kernel_func(int dtype);
size_t batch_list_lds_bytes(int list);
const void* batch_list_func(int list);
hipError_t launch_batch_list(int list, const void* in, void* out, const void* lt, const int64_t* offs,
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
