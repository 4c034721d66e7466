// binary32 instantiations of the FFT kernels.
#include "fft_device.hpp"
#define ELEM_T f2_t
#define DTYPE_ID DT_F32
#define TABLE_FN kernel_table_f32
#include "kernels_inst.hpp"
