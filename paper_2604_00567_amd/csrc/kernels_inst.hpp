// Instantiates every configuration of configs.inc for one element type
// (included by kernels_f16.hip / kernels_f32.hip with ELEM_T, DTYPE_ID, TABLE_FN).
#include "fft_device.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace dsfft {

// The kernel entry for a configuration: the pipelined entry (with its
// occupancy attribute) only where PIPE = 1.
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE>
static constexpr auto kernel_entry() {
    if constexpr (PIPE == 1)
        return &fft_unit_kernel_pipe<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>;
    else
        return &fft_unit_kernel<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>;
}

template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE>
static hipError_t launch_unit(const void* in, void* out, const void* lt, int64_t units, int log_m,
                              hipStream_t stream) {
    using TW = typename TwOf<E>::type;
    constexpr int NT = (UPW / UPL) << (LOG_NU - LOG_E);
    constexpr size_t LDS =
        (size_t)UPW * PassPlan<LOG_NU, LR0, LR1, LR2, LANE>::region() * sizeof(E);
    auto kern = kernel_entry<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>();
    int64_t grid = (units + UPW - 1) / UPW;
    if (grid <= 0) return hipSuccess;
    if (PIPE == 1) {
        // persistent grid: the workgroups that fit on the device at once
        static int resident = 0;
        if (!resident) {
            int dev = 0, cus = 0, per = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, NT, LDS) != hipSuccess)
                return hipErrorInvalidConfiguration;
            resident = cus * (per > 0 ? per : 1);
        }
        grid = grid < resident ? grid : resident;
    }
    if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), LDS, stream, (const E*)in, (E*)out,
                       (const TW*)lt, units, log_m);
    return hipGetLastError();
}

#define CFGU(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, UPL)                   \
    {DTYPE_ID, MODE, LOG_NU, LOG_E, UPW, UPL, {LR0, LR1, LR2}, STG, LANE, PIPE,                \
     ((UPW) / (UPL)) << ((LOG_NU) - (LOG_E)),                                                  \
     (size_t)(UPW) * PassPlan<LOG_NU, LR0, LR1, LR2, LANE>::region() * sizeof(ELEM_T),         \
     &launch_unit<ELEM_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>,      \
     (const void*)kernel_entry<ELEM_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE,   \
                               PIPE>()},
#define CFG(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE)                          \
    CFGU(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, 1)

static const KernelCfg kTable[] = {
#include "configs.inc"
};
#undef CFG
#undef CFGU

const KernelCfg* TABLE_FN(int* count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dsfft
