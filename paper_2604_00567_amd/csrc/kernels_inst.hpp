// Instantiates every configuration of configs.inc for one element type
// (included by kernels_f16.hip / kernels_f32.hip with ELEM_T, DTYPE_ID, TABLE_FN).
#include "fft_device.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace dsfft {

template <class E, int LOG_NU, int LOG_E, int UPW, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE>
static hipError_t launch_unit(const void* in, void* out, const void* lt, int64_t units, int log_m,
                              hipStream_t stream) {
    using TW = typename TwOf<E>::type;
    constexpr int NT = UPW << (LOG_NU - LOG_E);
    constexpr size_t LDS =
        (size_t)UPW * PassPlan<LOG_NU, LR0, LR1, LR2, LANE>::region() * sizeof(E);
    const int64_t grid = (units + UPW - 1) / UPW;
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((fft_unit_kernel<E, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE>),
                       dim3((unsigned)grid), dim3(NT), LDS, stream, (const E*)in, (E*)out,
                       (const TW*)lt, units, log_m);
    return hipGetLastError();
}

#define CFG(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE)                                \
    {DTYPE_ID, MODE, LOG_NU, LOG_E, UPW, {LR0, LR1, LR2}, STG, LANE,                           \
     (UPW) << ((LOG_NU) - (LOG_E)),                                                            \
     (size_t)(UPW) * PassPlan<LOG_NU, LR0, LR1, LR2, LANE>::region() * sizeof(ELEM_T),         \
     &launch_unit<ELEM_T, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE>,                 \
     (const void*)&fft_unit_kernel<ELEM_T, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE>},

static const KernelCfg kTable[] = {
#include "configs.inc"
};
#undef CFG

const KernelCfg* TABLE_FN(int* count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dsfft
