// Instantiates every configuration of configs.inc for one element type
// (included by kernels_f16.hip / kernels_f32.hip with ELEM_T, DTYPE_ID, TABLE_FN).
#include "fft_device.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace dsfft {

// Whether the configuration fits a workgroup's LDS with element type E.
template <class E, int LOG_NU, int LOG_E, int UPW, int MODE, int LR0, int LR1, int LR2, int LANE>
static constexpr bool cfg_fits() {
    return unit_fits<E, LOG_E, MODE, UPW, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>>();
}

// The kernel of a configuration: the pipelined entry (with its occupancy
// attribute) only where PIPE = 1.
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE>
static constexpr auto kernel_ptr() {
    if constexpr (PIPE == 1)
        return &fft_unit_kernel_pipe<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>;
    else
        return &fft_unit_kernel<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>;
}

// Its entry for the registry; none for a configuration that does not fit
// (that kernel is not instantiated).
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE>
static constexpr const void* kernel_entry() {
    if constexpr (!cfg_fits<E, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, LANE>())
        return nullptr;
    else
        return (const void*)kernel_ptr<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>();
}

template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE>
static hipError_t launch_unit(const void* in, void* out, const void* lt, int64_t units, int log_m,
                              hipStream_t stream) {
    using TW = typename TwOf<E>::type;
    if constexpr (!cfg_fits<E, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, LANE>()) {
        return hipErrorInvalidConfiguration;
    } else {
    constexpr int NT = (UPW / UPL) << (LOG_NU - LOG_E);
    constexpr size_t LDS =
        unit_lds_elems<E, LOG_E, MODE, UPW, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>>() * sizeof(E);
    auto kern = kernel_ptr<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>();
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
}

// An entry that does not fit gets mode -1: no plan or tuner ever selects it.
#define CFGU(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, UPL)                   \
    {DTYPE_ID,                                                                                 \
     cfg_fits<ELEM_T, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, LANE>() ? (MODE) : -1,          \
     LOG_NU, LOG_E, UPW, UPL, {LR0, LR1, LR2}, STG, LANE, PIPE,                                 \
     ((UPW) / (UPL)) << ((LOG_NU) - (LOG_E)),                                                  \
     unit_lds_elems<ELEM_T, LOG_E, MODE, UPW, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>>() *        \
         sizeof(ELEM_T),                                                                       \
     &launch_unit<ELEM_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>,      \
     kernel_entry<ELEM_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE>()},
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
