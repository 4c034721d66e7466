// binary16 instantiations of the FFT kernels.
#include <stdint.h>
#define ELEM_T uint32_t
#define DTYPE_ID DT_F16
#define TABLE_FN kernel_table_f16
#include "kernels_inst.hpp"
