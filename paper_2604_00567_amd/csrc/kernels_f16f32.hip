// Instantiations with binary16 storage and binary32 butterflies: inputs and
// outputs are binary16 pairs, widened exactly on load and rounded once (to
// nearest even) on store; every pass, the LDS exchanges and the two-pass
// intermediate are binary32, with the binary32 table.
#include "fft_device.hpp"
#define ELEM_T f2_t
#define STORE_T uint32_t
#define DTYPE_ID DT_F16F32
#define TABLE_FN kernel_table_f16f32
#include "kernels_inst.hpp"
