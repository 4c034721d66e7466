// Registry of compiled kernel configurations (one entry per template
// instantiation of fft_unit_kernel).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dsfft {

typedef hipError_t (*LaunchFn)(const void* in, void* out, const void* lt, int64_t units,
                               int log_m, hipStream_t stream);

struct KernelCfg {
    int dtype;      // DT_F16 / DT_F32 / DT_F16F32
    int mode;       // MODE_SMALL / MODE_COLS / MODE_ROWS
    int log_nu;     // unit size (log2)
    int log_e;      // elements per lane and unit (log2)
    int upw;        // units per workgroup
    int upl;        // units per lane (a lane's groups of one position in UPL units)
    int lr[3];      // register-pass radices (log2; 0 = absent)
    int staged;     // 1: block copied through LDS with 16-byte accesses
    int lane_tail;  // 1: the last two stages run across lanes (permlane swaps)
    int pipelined;  // 1: persistent workgroups prefetch the next block into registers;
                    // 2: each pass loads the next pass's twiddles
    int encoding;   // path encoding of the butterfly: 0 table, 1 select, 2 branch
    int threads;    // workgroup size
    size_t lds_bytes;
    LaunchFn launch;
    const void* func;
};

// All configurations for one dtype, in order of preference per (mode, log_nu).
const KernelCfg* kernel_table_f16(int* count);
const KernelCfg* kernel_table_f32(int* count);
const KernelCfg* kernel_table_f16f32(int* count);

}  // namespace dsfft
