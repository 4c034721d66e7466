// Host-side twiddle tables (Algorithm 1 of arXiv 2604.00567 and the two
// single-factorisation baselines), generated in FP64 with the C library's
// cos/sin, rounded once to the plan's precision, and laid out for the device.
#include "tables.hpp"

#include <cmath>
#include <cstring>

namespace dsfft {

static constexpr double kEpsClamp = 1e-7;   // Linzer-Feig clamp of sin(theta)

// Entry k of the size-n table in FP64.  theta = -(2 pi k)/n, w_r = cos, w_i = sin;
// for the inverse transform the twiddle is the conjugate W^{-k} = (w_r, -w_i)
// and the same rules below apply to it.
//   dual-select (Algorithm 1): |w_r| >= |w_i| -> (w_r, w_i/w_r, cosine path),
//                              else (w_i, w_r/w_i, sine path);   |ratio| <= 1.
//   Linzer-Feig (Sec. II-B):   (w_i', w_r/w_i', sine) with w_i' = +1e-7 if |w_i| < 1e-7.
//   cosine (Sec. II-C):        (w_r, w_i/w_r, cosine).
//   Linzer-Feig, W^0 exempt:   k = 0 on the cosine path, the rest Linzer-Feig.
Twiddle64 twiddle64(int64_t k, int64_t n, int kind, bool inverse) {
    const double angle = -((2.0 * M_PI) * (double)k) / (double)n;
    const double wr = std::cos(angle), wi = inverse ? -std::sin(angle) : std::sin(angle);
    bool cos_path;
    switch (kind) {
        case TABLE_DUAL_SELECT: cos_path = std::fabs(wr) >= std::fabs(wi); break;
        case TABLE_COSINE: cos_path = true; break;
        case TABLE_LF_W0_EXEMPT: cos_path = (k == 0); break;
        default: cos_path = false; break;
    }
    Twiddle64 t;
    if (cos_path) {
        t.mult = wr;
        t.ratio = wi / wr;
        t.sine = false;
    } else {
        double d = wi;
        if (kind == TABLE_LINZER_FEIG && std::fabs(d) < kEpsClamp) d = kEpsClamp;
        t.mult = d;
        t.ratio = wr / d;
        t.sine = true;
    }
    return t;
}

// IEEE binary64 -> binary16, round to nearest, ties to even, working on the
// bit pattern (53-bit significand shifted down to 11 or fewer bits).
uint16_t f64_to_f16(double x) {
    uint64_t bits;
    std::memcpy(&bits, &x, 8);
    const uint16_t sign = (uint16_t)((bits >> 48) & 0x8000u);
    const int bexp = (int)((bits >> 52) & 0x7ff);
    const uint64_t frac = bits & 0xFFFFFFFFFFFFFull;
    if (bexp == 0x7ff) return (uint16_t)(sign | 0x7c00u | (frac ? 0x0200u : 0u));
    if (bexp == 0) return sign;                       // FP64 subnormals are far below 2^-25
    const int e = bexp - 1023;
    if (e > 15) return (uint16_t)(sign | 0x7c00u);
    const uint64_t sig = frac | (1ull << 52);
    int drop;
    uint32_t hexp;
    if (e >= -14) {
        drop = 42;
        hexp = (uint32_t)(e + 15);
    } else {
        drop = 42 + (-14 - e);
        hexp = 0;
        if (drop > 63) return sign;
    }
    uint64_t q = sig >> drop;
    const uint64_t rem = sig & ((1ull << drop) - 1);
    const uint64_t halfway = 1ull << (drop - 1);
    if (rem > halfway || (rem == halfway && (q & 1))) ++q;
    uint32_t out = hexp == 0 ? (uint32_t)q : ((hexp << 10) + (uint32_t)(q - 1024));
    if (out >= 0x7c00u) out = 0x7c00u;
    return (uint16_t)(sign | out);
}

static inline uint32_t f32_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

// Device entry for one twiddle (layouts in fft_device.hpp: TwH / TwF).
static void pack_entry(const Twiddle64& t, int dtype, uint8_t* dst) {
    if (dtype == DT_F16) {
        const uint16_t m = f64_to_f16(t.mult);
        const uint16_t r = f64_to_f16(t.ratio);
        const uint16_t sm = t.sine ? (uint16_t)(m ^ 0x8000u) : m;
        const uint32_t w = (uint32_t)sm | ((uint32_t)m << 16);
        const uint32_t ts = (t.sine ? 16u : 0u) | ((uint32_t)r << 16);
        std::memcpy(dst, &w, 4);
        std::memcpy(dst + 4, &ts, 4);
    } else {
        const float m = (float)t.mult;
        const float r = (float)t.ratio;
        const float sm = t.sine ? -m : m;
        const uint32_t mask = t.sine ? 0xFFFFFFFFu : 0u;
        std::memcpy(dst, &sm, 4);
        std::memcpy(dst + 4, &m, 4);
        std::memcpy(dst + 8, &r, 4);
        std::memcpy(dst + 12, &mask, 4);
    }
}

size_t entry_bytes(int dtype) { return dtype == DT_F16 ? 8 : 16; }

std::vector<uint8_t> build_level_table(int64_t ncap, int dtype, int kind, bool inverse) {
    const size_t eb = entry_bytes(dtype);
    std::vector<uint8_t> img((size_t)ncap * eb, 0);
    for (int64_t L = 2; L <= ncap; L <<= 1)
        for (int64_t j = 0; j < L / 2; ++j)
            pack_entry(twiddle64(j, L, kind, inverse), dtype, img.data() + (size_t)(L / 2 + j) * eb);
    return img;
}

Radix4Entry radix4_entry(int64_t j, int64_t L, int kind, bool inverse) {
    Radix4Entry e;
    for (int p = 0; p < 3; ++p) e.w[p] = twiddle64((p + 1) * j, L, kind, inverse);
    const double m1 = e.w[0].mult, m3 = e.w[2].mult;
    e.sel = std::fabs(m1) >= std::fabs(m3);
    e.rho = e.sel ? m3 / m1 : m1 / m3;
    return e;
}

size_t entry4_bytes(int dtype) { return dtype == DT_F16 ? 32 : 64; }

static inline uint32_t pack_h2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }
static inline uint16_t neg16(uint16_t h) { return (uint16_t)(h ^ 0x8000u); }

// One radix-4 device entry.  Signs: sigma = -1 on the sine path; sigma_M is
// the outer multiplier's; sg = +1 when the outer multiplier is m(W^j).  The
// inverse stores the last multiplier pair negated (Y1 and Y3 trade places).
static void pack_entry4(const Radix4Entry& e, int dtype, bool inverse, uint8_t* dst) {
    const bool s1 = e.w[0].sine, s2 = e.w[1].sine, s3 = e.w[2].sine;
    const bool sM = e.sel ? s1 : s3;
    const bool flip13 = s1 != s3;          // sigma1 sigma3 = -1
    const bool neg_mm1 = (!e.sel) != inverse;
    const double M64 = e.sel ? e.w[0].mult : e.w[2].mult;
    if (dtype == DT_F16) {
        uint32_t wd[8];
        for (int p = 0; p < 3; ++p)
            wd[p] = (e.w[p].sine ? 16u : 0u) | ((uint32_t)f64_to_f16(e.w[p].ratio) << 16);
        const uint16_t m2 = f64_to_f16(e.w[1].mult);
        wd[3] = pack_h2(s2 ? neg16(m2) : m2, m2);
        const uint16_t rho = f64_to_f16(e.rho);
        wd[4] = pack_h2(flip13 ? neg16(rho) : rho, rho);
        const uint16_t M = f64_to_f16(M64);
        const uint16_t sm = sM ? neg16(M) : M;      // sigma_M M
        wd[5] = pack_h2(sm, M);
        // (sg M, -sg sigma_M M), negated for the inverse
        uint16_t a = M, b = neg16(sm);
        if (neg_mm1) {
            a = neg16(a);
            b = neg16(b);
        }
        wd[6] = pack_h2(a, b);
        wd[7] = e.sel ? 0xFFFFFFFFu : 0u;
        std::memcpy(dst, wd, sizeof wd);
    } else {
        float f[16];
        uint32_t u[16];
        for (int p = 0; p < 3; ++p) {
            f[p] = (float)e.w[p].ratio;
            u[3 + p] = e.w[p].sine ? 0xFFFFFFFFu : 0u;
        }
        const float m2 = (float)e.w[1].mult;
        f[6] = s2 ? -m2 : m2;
        f[7] = m2;
        const float rho = (float)e.rho;
        f[8] = flip13 ? -rho : rho;
        f[9] = rho;
        const float M = (float)M64;
        const float sm = sM ? -M : M;
        f[10] = sm;
        f[11] = M;
        f[12] = neg_mm1 ? -M : M;
        f[13] = neg_mm1 ? sm : -sm;
        for (int i = 0; i < 3; ++i) std::memcpy(&u[i], &f[i], 4);
        for (int i = 6; i < 14; ++i) std::memcpy(&u[i], &f[i], 4);
        u[14] = e.sel ? 0xFFFFFFFFu : 0u;
        u[15] = 0;
        std::memcpy(dst, u, sizeof u);
    }
}

// Entry 0: the radix-2 butterfly of W^0 (span 2) in the fields the radix-2
// stage reads (ts1 and w2 / t1, mask1, sm2 and m2).
static void pack_w0_entry4(const Twiddle64& t, int dtype, uint8_t* dst) {
    uint8_t r2[16];
    pack_entry(t, dtype, r2);
    if (dtype == DT_F16) {
        std::memcpy(dst + 0, r2 + 4, 4);    // ts1 <- ts
        std::memcpy(dst + 12, r2 + 0, 4);   // w2 <- w
    } else {
        std::memcpy(dst + 24, r2 + 0, 8);   // (sm2, m2) <- (sm, m)
        std::memcpy(dst + 0, r2 + 8, 4);    // t1 <- t
        std::memcpy(dst + 12, r2 + 12, 4);  // mask1 <- mask
    }
}

std::vector<uint8_t> build_level_table4(int64_t ncap, int dtype, int kind, bool inverse) {
    const size_t eb = entry4_bytes(dtype);
    // ncap entries, the upper half unused: a radix-R pass of span L0 R reads
    // entries below L0 R / 2, and LDS copies of a pass's run [L0, L0 R) stay
    // inside the image
    std::vector<uint8_t> img((size_t)ncap * eb, 0);
    pack_w0_entry4(twiddle64(0, 2, kind, inverse), dtype, img.data());
    for (int64_t L = 4; L <= ncap; L <<= 1)
        for (int64_t j = 0; j < L / 4; ++j)
            pack_entry4(radix4_entry(j, L, kind, inverse), dtype, inverse,
                        img.data() + (size_t)(L / 4 + j) * eb);
    return img;
}

static void store_rounded(int dtype, double v, void* out, int64_t i) {
    if (!out) return;
    if (dtype == DT_F16) {
        const uint16_t h = f64_to_f16(v);
        std::memcpy((uint8_t*)out + 2 * i, &h, 2);
    } else {
        const uint32_t u = f32_bits((float)v);
        std::memcpy((uint8_t*)out + 4 * i, &u, 4);
    }
}

void build_flat_table4(int64_t n, int dtype, int kind, bool inverse, void* mult, void* ratio,
                       uint8_t* path, void* rho, uint8_t* sel) {
    for (int64_t k = 0; k < 3 * n / 4; ++k) {
        const Twiddle64 t = twiddle64(k, n, kind, inverse);
        store_rounded(dtype, t.mult, mult, k);
        store_rounded(dtype, t.ratio, ratio, k);
        if (path) path[k] = t.sine ? 1 : 0;
    }
    for (int64_t j = 0; j < n / 4; ++j) {
        const Radix4Entry e = radix4_entry(j, n, kind, inverse);
        store_rounded(dtype, e.rho, rho, j);
        if (sel) sel[j] = e.sel ? 1 : 0;
    }
}

void build_flat_table(int64_t n, int dtype, int kind, bool inverse, void* mult, void* ratio,
                      uint8_t* path) {
    for (int64_t k = 0; k < n / 2; ++k) {
        const Twiddle64 t = twiddle64(k, n, kind, inverse);
        if (dtype == DT_F16) {
            const uint16_t m = f64_to_f16(t.mult), r = f64_to_f16(t.ratio);
            if (mult) std::memcpy((uint8_t*)mult + 2 * k, &m, 2);
            if (ratio) std::memcpy((uint8_t*)ratio + 2 * k, &r, 2);
        } else {
            const uint32_t m = f32_bits((float)t.mult), r = f32_bits((float)t.ratio);
            if (mult) std::memcpy((uint8_t*)mult + 4 * k, &m, 4);
            if (ratio) std::memcpy((uint8_t*)ratio + 4 * k, &r, 4);
        }
        if (path) path[k] = t.sine ? 1 : 0;
    }
}

}  // namespace dsfft
