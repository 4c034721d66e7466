// Instantiates every configuration of configs.inc for one element type
// (included by kernels_f16.hip / kernels_f32.hip / kernels_f16f32.hip with
// ELEM_T (compute type), STORE_T (storage type of the plan's input and
// output, ELEM_T if not defined), DTYPE_ID and TABLE_FN).
#include <type_traits>

#include "fft_device.hpp"
#include "kernels.hpp"
#include "tables.hpp"

#ifndef STORE_T
#define STORE_T ELEM_T
#endif

namespace dsfft {

// Input and output storage of a kernel computing in E for a plan stored in
// S: whole transforms read and write S; the two-pass schedule keeps its
// intermediate in E (columns read S and write E, rows read E and write S).
template <class E, class S, int MODE>
struct IoOf {
    using in = std::conditional_t<MODE == MODE_ROWS, E, S>;
    using out = std::conditional_t<MODE == MODE_COLS, E, S>;
};

// Whether a configuration is compiled for (E, S): it fits a workgroup's LDS,
// with S != E it is not pipelined, nor staged with the lane tail (whose
// 16-byte copies move stored values unchanged), and a path encoding other than the table's is a
// binary16 variant of a plain kernel.
template <class E, class S, int LOG_NU, int LOG_E, int UPW, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE, int ENC>
static constexpr bool cfg_fits() {
    if constexpr (!std::is_same_v<E, S>)
        if ((STG && LANE) || PIPE == 1) return false;
    // the radix-4 form: whole transforms stored as computed, no lane tail, no
    // second register set or prefetch, passes on radix-4 stage boundaries
    if (ENC == ENC_RADIX4) {
        if (!std::is_same_v<E, S> || MODE != MODE_SMALL || LANE || PIPE == 1 || PIPE == 2 || PIPE == 5)
            return false;
        if (LR0 % 2 != LOG_NU % 2 || LR1 % 2 || LR2 % 2) return false;
    } else if (ENC != ENC_TABLE &&
               (!std::is_same_v<E, uint32_t> || !std::is_same_v<E, S> || PIPE == 1 || LANE)) {
        // the path-encoding variants: binary16 plans, plain (non-pipelined, no lane tail) kernels
        return false;
    }
    // staged blocks pass through the whole exchange area, which a two-round
    // exchange halves
    if (STG && exchange_rounds<E, LOG_E, MODE, UPW, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>>() == 2) return false;
    return unit_fits<E, LOG_NU, LOG_E, MODE, UPW, LANE, PIPE, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>, ENC>();
}

// The kernel of a configuration: the pipelined entry (with its occupancy
// attribute) only where PIPE = 1.
template <class E, class S, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2,
          int STG, int LANE, int PIPE, int ENC>
static constexpr auto kernel_ptr() {
    using IO = IoOf<E, S, MODE>;
    if constexpr (PIPE == 1)
        return &fft_unit_kernel_pipe<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE,
                                     typename IO::in, typename IO::out, ENC>;
    else
        return &fft_unit_kernel<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE,
                                typename IO::in, typename IO::out, ENC>;
}

// Its entry for the registry; none for a configuration that is not compiled.
template <class E, class S, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2,
          int STG, int LANE, int PIPE, int ENC>
static constexpr const void* kernel_entry() {
    if constexpr (!cfg_fits<E, S, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>())
        return nullptr;
    else
        return (const void*)kernel_ptr<E, S, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE,
                                       ENC>();
}

template <class E, class S, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2,
          int STG, int LANE, int PIPE, int ENC>
static hipError_t launch_unit(const void* in, void* out, const void* lt, int64_t units, int log_m,
                              hipStream_t stream) {
    using TW = TwT<E, ENC>;
    using IO = IoOf<E, S, MODE>;
    if constexpr (!cfg_fits<E, S, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>()) {
        return hipErrorInvalidConfiguration;
    } else {
        constexpr int NT = (UPW / UPL) << (LOG_NU - LOG_E);
        constexpr size_t LDS =
            unit_lds_bytes<E, LOG_NU, LOG_E, MODE, UPW, LANE, PIPE, PassPlan<LOG_NU, LR0, LR1, LR2, LANE>, ENC>();
        auto kern = kernel_ptr<E, S, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>();
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
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), LDS, stream, (const typename IO::in*)in,
                           (typename IO::out*)out, (const TW*)lt, units, log_m);
        return hipGetLastError();
    }
}

// An entry that is not compiled gets mode -1: no plan or tuner ever selects it.
#define CFGE(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, UPL, ENC)              \
    {DTYPE_ID,                                                                                 \
     cfg_fits<ELEM_T, STORE_T, LOG_NU, LOG_E, UPW, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>() \
         ? (MODE)                                                                              \
         : -1,                                                                                 \
     LOG_NU, LOG_E, UPW, UPL, {LR0, LR1, LR2}, STG, LANE, PIPE, ENC,                            \
     ((UPW) / (UPL)) << ((LOG_NU) - (LOG_E)),                                                  \
     unit_lds_bytes<ELEM_T, LOG_NU, LOG_E, MODE, UPW, LANE, PIPE,                               \
                    PassPlan<LOG_NU, LR0, LR1, LR2, LANE>, ENC>(),                             \
     &launch_unit<ELEM_T, STORE_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>, \
     kernel_entry<ELEM_T, STORE_T, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE, ENC>()},
#define CFGU(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, UPL)                   \
    CFGE(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, UPL, ENC_TABLE)
#define CFG(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE)                          \
    CFGU(MODE, LOG_NU, LOG_E, UPW, LR0, LR1, LR2, STG, LANE, PIPE, 1)

static const KernelCfg kTable[] = {
#include "configs.inc"
};
#undef CFG
#undef CFGU
#undef CFGE

const KernelCfg* TABLE_FN(int* count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace dsfft
