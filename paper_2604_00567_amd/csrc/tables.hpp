// Host-side twiddle tables: FP64 generation (Algorithm 1 and the baselines),
// single rounding to binary16/binary32, and the level-ordered device image.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace dsfft {

// DT_F16F32: binary16 storage, binary32 butterflies and table.
enum { DT_F16 = 0, DT_F32 = 1, DT_F16F32 = 2 };
// The table (and arithmetic) precision of a plan dtype.
inline int table_dtype(int dtype) { return dtype == DT_F16 ? DT_F16 : DT_F32; }
enum { TABLE_DUAL_SELECT = 0, TABLE_LINZER_FEIG = 1, TABLE_COSINE = 2, TABLE_LF_W0_EXEMPT = 3 };

struct Twiddle64 {
    double mult;
    double ratio;
    bool sine;     // false: cosine factorisation, true: sine factorisation
};

Twiddle64 twiddle64(int64_t k, int64_t n, int kind, bool inverse);
uint16_t f64_to_f16(double x);
size_t entry_bytes(int dtype);

// Device image with entry L/2 + j = T_L[j] for L = 2 .. ncap (entry 0 unused);
// `inverse`: the tables of the inverse transform (conjugate twiddles).
// Device tables are built for ncap >= kMinTableEntries, so kernels may copy
// that many leading entries whatever sizes their plan or batch holds.
constexpr int64_t kMinTableEntries = 4096;
std::vector<uint8_t> build_level_table(int64_t ncap, int dtype, int kind, bool inverse);

// Flat table T_n[k], k < n/2: rounded mult and ratio (binary16 bits or float)
// and the path byte (0 cosine, 1 sine).  Null outputs are skipped.
void build_flat_table(int64_t n, int dtype, int kind, bool inverse, void* mult, void* ratio,
                      uint8_t* path);

}  // namespace dsfft
