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

// Radix-4 form (Sec. VI, generality): the butterfly of span L and column j
// uses the entries of W_L^j, W_L^2j and W_L^3j (3j may reach 3L/4) and the
// odd pair's choice: sel = |m(W^j)| >= |m(W^3j)| on the FP64 multipliers, and
// rho = smaller/larger multiplier in FP64, rounded once.
struct Radix4Entry {
    Twiddle64 w[3];   // W^j, W^2j, W^3j
    bool sel;         // outer multiplier m(W^j) (else m(W^3j))
    double rho;
};
Radix4Entry radix4_entry(int64_t j, int64_t L, int kind, bool inverse);
size_t entry4_bytes(int dtype);
// Device image of the radix-4 table (layouts Tw4H / Tw4F in fft_device.hpp):
// entry L/4 + j for L = 4 .. ncap, j < L/4, and entry 0 = the radix-2 entry
// of W^0 for the span-2 stage of odd log2 N; ncap entries (the upper half zero).
std::vector<uint8_t> build_level_table4(int64_t ncap, int dtype, int kind, bool inverse);
// Flat radix-4 export for size n: rounded mult / ratio / path of W^k for
// k < 3n/4 (as build_flat_table), and per column j < n/4 of the last stage the
// rounded rho and sel byte.  Null outputs are skipped.
void build_flat_table4(int64_t n, int dtype, int kind, bool inverse, void* mult, void* ratio,
                       uint8_t* path, void* rho, uint8_t* sel);

// Flat table T_n[k], k < n/2: rounded mult and ratio (binary16 bits or float)
// and the path byte (0 cosine, 1 sine).  Null outputs are skipped.
void build_flat_table(int64_t n, int dtype, int kind, bool inverse, void* mult, void* ratio,
                      uint8_t* path);

}  // namespace dsfft
