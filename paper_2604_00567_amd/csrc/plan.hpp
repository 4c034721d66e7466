// Plan object and internal helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>

#include "kernels.hpp"

namespace dsfft {

struct DeviceTable {
    void* ptr = nullptr;
    int64_t ncap = 0;
    size_t bytes = 0;
    ~DeviceTable();
};

int set_error(int code, const std::string& msg);
int hip_error(hipError_t e, const char* where);
// The shared device table of (device, dtype, kind, direction, radix) covering
// size n (radix 2: level-ordered radix-2 entries; radix 4: the radix-4 form's).
int get_table(int64_t n, int dtype, int kind, bool inverse, std::shared_ptr<DeviceTable>* out,
              int radix = 2);
// The variant-th compiled configuration of (dtype, mode, log_nu) among those
// of the radix-2 butterflies (radix4 = false) or of the radix-4 form.
const KernelCfg* find_kernel(int dtype, int mode, int log_nu, int variant, bool radix4 = false);
int count_kernels(int dtype, int mode, int log_nu, bool radix4 = false);
std::string describe(const KernelCfg* k);
int elem_bytes(int dtype);
int work_elem_bytes(int dtype);

}  // namespace dsfft

struct fft_plan {
    int64_t n = 0, batch = 0;
    int log_n = 0, dtype = 0, kind = 0, device = 0;
    bool inverse = false;                   // inverse transform (conjugate tables)
    int radix = 2;                          // 4: the radix-4 form (radix-4 table and kernels)
    std::shared_ptr<dsfft::DeviceTable> table;
    const dsfft::KernelCfg* k1 = nullptr;   // single kernel, or the column kernel
    const dsfft::KernelCfg* k1_plain = nullptr;  // k1's size without 16-byte staging
    const dsfft::KernelCfg* k2 = nullptr;   // row kernel of the two-pass schedule
    int64_t chunk = 0;                      // transforms per two-pass chunk
    size_t ws_need = 0, ws_bytes = 0;
    void* ws = nullptr;
    bool ws_owned = false;
    ~fft_plan();
};

namespace dsfft {
// alloc_ws = false: a two-pass plan gets no workspace of its own (the caller
// sets one before the first execute).
fft_plan* plan_create(int64_t n, int64_t batch, int dtype, int kind, const int* variants,
                      bool inverse = false, int radix = 2, bool alloc_ws = true);
// Largest workspace a two-pass plan asks for (its chunk cap).
constexpr size_t kMaxWorkspaceBytes = (size_t)128 << 20;
bool tuned_choice(int dtype, int log_n, int* variants);
int plan_execute(fft_plan* p, const void* in, void* out, hipStream_t s);
// Frees a plan-owned workspace after the plan's device is idle.
void release_workspace(fft_plan* p);
// Argument checks of an execute (null, alignment, partial overlap).
int check_execute_args(const fft_plan* p, const void* in, const void* out);
// The plan's launches with its two-pass intermediate in ws, chunk transforms at a time.
int launch_plan_ws(const fft_plan* p, const void* in, void* out, hipStream_t s, void* ws, int64_t chunk);
}  // namespace dsfft
