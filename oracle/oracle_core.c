/*
 * Oracle core: a plain, slow, obviously correct CPU implementation of what the
 * dual-select FFT path computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table generator or constant with the HIP library, and the HIP
 * library never loads it.
 *
 * Paper: M. A. Bergach, "Dual-Select FMA Butterfly for FFT: Eliminating Twiddle
 * Factor Singularities with Bounded Precomputed Ratios" (arXiv 2604.00567).
 *
 * Contents
 *   - twiddle tables in FP64: dual-select (Algorithm 1), epsilon-clamped
 *     Linzer-Feig (Sec. II-B plus the clamp named in the introduction), pure
 *     cosine (Sec. II-C), and Linzer-Feig with W^0 exempted (a reading used to
 *     give the 163-ratio table a finite FP16 counterpart);
 *   - the FP64 reference: the DFT of eq. (1) written out (O(N^2)), and a plain
 *     radix-2 Stockham FFT with the 10-flop butterfly of eqs. (std1)-(std2);
 *   - the low-precision emulation: the same radix-2 Stockham pass order, every
 *     butterfly done as the six FMAs of eqs. (lf-s)-(lf-B) or (berg-s)-(berg-B),
 *     each FMA rounded once to the working precision (FP16, FP32, or FP64);
 *   - a direct double -> binary16 round-to-nearest-even conversion.
 *
 * The inverse transform (x[n] = sum_k X[k] W^{-nk}, unnormalised) uses the
 * conjugate twiddles W^{-k} = (w_r, -w_i); its tables follow the same rules
 * (selection, clamp) applied to them.  The paper names only the round trip
 * (Sec. V, binary32 relative L2 of about 1e-7); the inverse it implies is
 * this one.
 *
 * Readings taken where the paper is silent or misprinted:
 *   - theta = -(2*pi*k)/N evaluated in FP64 in that order (Algorithm 1 does not
 *     fix the order); cos/sin from the C library.
 *   - Sec. II-B prints s2 = cot(theta)*b_r + b_i; that does not reconstruct W*b.
 *     The factorisation identity ax+by = a(x+(b/a)y) applied to
 *     A_i = a_i + (w_i b_r + w_r b_i) gives s2 = b_r + cot(theta)*b_i, which is
 *     what is used here (the tests show the printed form fails the DFT).
 *   - the Linzer-Feig clamp replaces w_i by +1e-7 when |w_i| < 1e-7.
 *   - the FFT is forward and unnormalised, X[k] = sum_n x[n] W^{nk}.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { K_DUAL_SELECT = 0, K_LINZER_FEIG = 1, K_COSINE = 2, K_LF_W0_EXEMPT = 3 };
enum { P_COS = 0, P_SIN = 1 };

#define ORC_EPS_CLAMP 1e-7

/* Planted-mistake switch, used only by the test that shows the pins catch
 * plausible errors (built separately with -DORC_MUTANT=k; 0 in normal builds). */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

static int is_pow2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }
static int log2i(int64_t n) { int m = 0; while ((1LL << m) < n) ++m; return m; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Twiddle angle of W^k for size n (Sec. I: W = exp(-j 2 pi k / N)). */
double orc_theta(int64_t k, int64_t n) {
    double two_pi = 2.0 * M_PI;
    return -(two_pi * (double)k) / (double)n;
}

/*
 * Twiddle table for k in [0, n/2): multiplier, ratio and path per entry.
 *   dual-select (Algorithm 1): if |w_r| >= |w_i| take the cosine factorisation
 *       (w_r, w_i/w_r, COS), else the sine one (w_i, w_r/w_i, SIN);
 *   Linzer-Feig (Sec. II-B): (w_i', w_r/w_i', SIN) with w_i' = +eps when |w_i|<eps;
 *   cosine (Sec. II-C): (w_r, w_i/w_r, COS);
 *   Linzer-Feig with W^0 exempted: the k = 0 entry takes the cosine form, all
 *       others are Linzer-Feig.
 * Returns 0, or -1 on a bad argument.
 */
static void table_entry(int64_t k, int64_t n, int kind, int inverse, double* mult, double* ratio,
                        int32_t* path) {
    double th = orc_theta(k, n);
    double wr = cos(th), wi = sin(th);
    if (inverse) wi = -wi;                  /* W^{-k}: the conjugate */
    int use_cos;
    if (kind == K_DUAL_SELECT) use_cos = fabs(wr) >= fabs(wi);
    else if (kind == K_COSINE) use_cos = 1;
    else if (kind == K_LF_W0_EXEMPT) use_cos = (k == 0);
    else use_cos = 0;
    if (use_cos) {
        *mult = wr;
        *ratio = wi / wr;
        *path = P_COS;
    } else {
        double d = wi;
        if (kind == K_LINZER_FEIG && fabs(d) < ORC_EPS_CLAMP) d = ORC_EPS_CLAMP;
        *mult = d;
        *ratio = wr / d;
        *path = P_SIN;
    }
}

int orc_table_dir(int64_t n, int kind, int inverse, double* mult, double* ratio, int32_t* path) {
    if (!is_pow2(n) || kind < 0 || kind > 3) return -1;
    for (int64_t k = 0; k < n / 2; ++k) table_entry(k, n, kind, inverse, &mult[k], &ratio[k], &path[k]);
    return 0;
}

int orc_table(int64_t n, int kind, double* mult, double* ratio, int32_t* path) {
    return orc_table_dir(n, kind, 0, mult, ratio, path);
}

/* ---------------------------------------------------------------- binary16 */

/* Round a double to the nearest binary16 value, ties to even, in one step. */
uint16_t orc_rn16(double x) {
    uint16_t sign = signbit(x) ? 0x8000u : 0u;
    double a = fabs(x);
    if (isnan(x)) return (uint16_t)(sign | 0x7e00u);
    if (isinf(a)) return (uint16_t)(sign | 0x7c00u);
    if (a < ldexp(1.0, -14)) {
        /* subnormal range: units of 2^-24; q may reach 1024 = smallest normal */
        double q = rint(ldexp(a, 24));
        return (uint16_t)(sign | (uint16_t)q);
    }
    int ex;
    frexp(a, &ex);            /* a in [2^(ex-1), 2^ex) */
    int e = ex - 1;           /* binary16 exponent, >= -14 */
    double q = rint(ldexp(a, 10 - e));   /* in [1024, 2048] */
    if (q >= 2048.0) { q = 1024.0; e += 1; }
    if (e > 15) return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | (uint16_t)((e + 15) << 10) | (uint16_t)(q - 1024.0));
}

double orc_f16_to_double(uint16_t h) {
    int s = (h >> 15) & 1, e = (h >> 10) & 31, f = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)f, -24);
    else if (e == 31) v = f ? NAN : INFINITY;
    else v = ldexp((double)(1024 + f), e - 25);
    return s ? -v : v;
}

void orc_rn16_array(int64_t count, const double* x, uint16_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_rn16(x[i]);
}

void orc_f16_to_double_array(int64_t count, const uint16_t* h, double* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_f16_to_double(h[i]);
}

/* One FMA rounded once to binary16: the product of two binary16 values is exact
 * in FP64, and for results inside the binary16 range the FP64 sum keeps every
 * bit that decides the binary16 rounding. */
double orc_fma16(double a, double b, double c) {
    return orc_f16_to_double(orc_rn16(fma(a, b, c)));
}

/* One FMA rounded once to binary32 (C99 fmaf is correctly rounded). */
float orc_fma32(float a, float b, float c) { return fmaf(a, b, c); }

/* --------------------------------------------------- the six-FMA butterfly */

/* precision of the emulation */
enum { PREC_F16 = 16, PREC_F32 = 32, PREC_F64 = 64 };

static inline double round_p(int prec, double x);

static inline double fma_p(int prec, double a, double b, double c) {
    if (ORC_MUTANT == 5 && prec == PREC_F16) return fma(a, b, c);
    if (ORC_MUTANT == 6 && prec != PREC_F64) return round_p(prec, round_p(prec, a * b) + c);
    if (prec == PREC_F16) return orc_fma16(a, b, c);
    if (prec == PREC_F32) return (double)fmaf((float)a, (float)b, (float)c);
    return fma(a, b, c);
}

static inline double round_p(int prec, double x) {
    if (prec == PREC_F16) return orc_f16_to_double(orc_rn16(x));
    if (prec == PREC_F32) return (double)(float)x;
    return x;
}

/*
 * A = a + W b, B = a - W b (eq. (1)) with W factorised by the table entry.
 * Cosine path, eqs. (berg-s)-(berg-B), t = tan(theta), m = cos(theta):
 *   s1 = b_r - t b_i        s2 = t b_r + b_i
 *   A_r = a_r + s1 m        A_i = a_i + s2 m
 *   B_r = a_r - s1 m        B_i = a_i - s2 m
 * Sine path, eqs. (lf-s)-(lf-B), t = cot(theta), m = sin(theta) (s2 as read
 * in the header):
 *   s1 = b_i - t b_r        s2 = b_r + t b_i
 *   A_r = a_r - s1 m        A_i = a_i + s2 m
 *   B_r = a_r + s1 m        B_i = a_i - s2 m
 * Every line is one FMA whose product is formed from the operands as printed
 * (a negated operand, never a negated result).
 */
static inline void bfly6(int prec, int path, double m, double t,
                         double ar, double ai, double br, double bi,
                         double* Ar, double* Ai, double* Br, double* Bi) {
    double s1, s2;
    if (path == P_COS) {
        s1 = fma_p(prec, -t, bi, br);
        s2 = fma_p(prec, t, br, bi);
        *Ar = fma_p(prec, ORC_MUTANT == 2 ? -s1 : s1, m, ar);
        *Ai = fma_p(prec, s2, m, ai);
        *Br = fma_p(prec, -s1, m, ar);
        *Bi = fma_p(prec, -s2, m, ai);
    } else {
        s1 = fma_p(prec, -t, br, bi);
        s2 = ORC_MUTANT == 1 ? fma_p(prec, t, br, bi) : fma_p(prec, t, bi, br);
        *Ar = fma_p(prec, -s1, m, ar);
        *Ai = fma_p(prec, s2, m, ai);
        *Br = fma_p(prec, s1, m, ar);
        *Bi = fma_p(prec, -s2, m, ai);
    }
}

/*
 * Radix-2 Stockham DIT over m = log2 N passes (Sec. IV-B assumes Stockham).
 * Y_0[r][0] = x[r]; for s = 1..m with L = 2^s, h = L/2, for r < N/L, j < h:
 *   a = Y_{s-1}[r][j], b = Y_{s-1}[r + N/L][j], twiddle W^(j N / L),
 *   Y_s[r][j] = A, Y_s[r][j + h] = B;
 * Y_s[r][q] lives at index r + (N/L) q, so Y_m[0][k] = X[k] in natural order.
 * y, z: work arrays of 2n doubles (interleaved re, im); result left in y.
 */
static void stockham_emulate(int64_t n, int prec, const double* mult, const double* ratio,
                             const int32_t* path, double* y, double* z) {
    int mlog = log2i(n);
    for (int s = 1; s <= mlog; ++s) {
        int64_t L = (int64_t)1 << s, h = L / 2, nl = n / L, nh = n / h;
        for (int64_t r = 0; r < nl; ++r) {
            for (int64_t j = 0; j < h; ++j) {
                int64_t k = ORC_MUTANT == 3 ? (j * nh) % (n / 2) : j * nl;
                int64_t ia = r + nh * j, ib = r + nl + nh * j;
                int64_t oa = r + nl * j, ob = r + nl * (j + h);
                double Ar, Ai, Br, Bi;
                if (ORC_MUTANT == 4) { int64_t tmp = ia; ia = ib; ib = tmp; }
                bfly6(prec, path[k], mult[k], ratio[k], y[2 * ia], y[2 * ia + 1],
                      y[2 * ib], y[2 * ib + 1], &Ar, &Ai, &Br, &Bi);
                z[2 * oa] = Ar; z[2 * oa + 1] = Ai;
                z[2 * ob] = Br; z[2 * ob + 1] = Bi;
            }
        }
        memcpy(y, z, sizeof(double) * 2 * (size_t)n);
    }
}

/* Table rounded once from FP64 to the working precision. */
static int rounded_table(int64_t n, int kind, int inverse, int prec, double** mult, double** ratio,
                         int32_t** path) {
    int64_t h = n / 2;
    *mult = (double*)malloc(sizeof(double) * h);
    *ratio = (double*)malloc(sizeof(double) * h);
    *path = (int32_t*)malloc(sizeof(int32_t) * h);
    if (!*mult || !*ratio || !*path) return -1;
    if (orc_table_dir(n, kind, inverse, *mult, *ratio, *path)) return -1;
    for (int64_t k = 0; k < h; ++k) {
        (*mult)[k] = round_p(prec, (*mult)[k]);
        (*ratio)[k] = round_p(prec, (*ratio)[k]);
    }
    return 0;
}

static int emulate_batch(int64_t n, int64_t batch, int kind, int inverse, int prec,
                         const double* in, double* out) {
    if (!is_pow2(n) || batch < 0) return -1;
    double *mult, *ratio; int32_t* path;
    if (rounded_table(n, kind, inverse, prec, &mult, &ratio, &path)) return -1;
    int err = 0;
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        if (!y || !z) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(static)
        for (int64_t b = 0; b < batch; ++b) {
            if (!y || !z) continue;
            for (int64_t i = 0; i < 2 * n; ++i) y[i] = round_p(prec, in[b * 2 * n + i]);
            stockham_emulate(n, prec, mult, ratio, path, y, z);
            memcpy(out + b * 2 * n, y, sizeof(double) * 2 * (size_t)n);
        }
        free(y); free(z);
    }
    free(mult); free(ratio); free(path);
    return err;
}

/* FP64 emulation of the six-FMA butterflies (each FMA rounded to FP64);
 * inverse != 0 runs the inverse transform (conjugate tables). */
int orc_emulate_f64(int64_t n, int64_t batch, int kind, int inverse, const double* in, double* out) {
    return emulate_batch(n, batch, kind, inverse, PREC_F64, in, out);
}

/* FP32 emulation: interleaved float in/out, each FMA rounded once to FP32. */
int orc_emulate_f32(int64_t n, int64_t batch, int kind, int inverse, const float* in, float* out) {
    size_t cnt = (size_t)(2 * n * batch);
    double* a = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    double* b = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    if (!a || !b) { free(a); free(b); return -1; }
    for (size_t i = 0; i < cnt; ++i) a[i] = (double)in[i];
    int rc = emulate_batch(n, batch, kind, inverse, PREC_F32, a, b);
    for (size_t i = 0; i < cnt && rc == 0; ++i) out[i] = (float)b[i];
    free(a); free(b);
    return rc;
}

/* FP16 emulation: interleaved binary16 bit patterns in/out. */
int orc_emulate_f16(int64_t n, int64_t batch, int kind, int inverse, const uint16_t* in, uint16_t* out) {
    size_t cnt = (size_t)(2 * n * batch);
    double* a = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    double* b = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    if (!a || !b) { free(a); free(b); return -1; }
    for (size_t i = 0; i < cnt; ++i) a[i] = orc_f16_to_double(in[i]);
    int rc = emulate_batch(n, batch, kind, inverse, PREC_F16, a, b);
    for (size_t i = 0; i < cnt && rc == 0; ++i) out[i] = orc_rn16(b[i]);
    free(a); free(b);
    return rc;
}

/* ------------------------------------------------- radix-4 butterflies */

/*
 * Radix-4 form of the method (Sec. VI, "Generality": in a radix-r butterfly
 * every twiddle multiplication picks its own min-ratio factorisation).
 *
 * Canonical order for N = 2^m: when m is odd, one radix-2 stage of span 2 (the
 * six-FMA butterfly with the W^0 entry) comes first; then radix-4 Stockham
 * DIT stages of span L = 4, 16, ... (m even) or 8, 32, ... (m odd) up to N.
 * A radix-4 stage of span L holds Y[r][q] at r + (N/L) q and, for r < N/L and
 * j < L/4, combines the four DFTs of span L/4 at residues r + p N/L:
 *   a = Y'[r][j], b = Y'[r + N/L][j], c = Y'[r + 2N/L][j], d = Y'[r + 3N/L][j]
 * (Y'[r'][j] at r' + (4N/L) j) with W1 = W^{jN/L}, W2 = W1^2, W3 = W1^3:
 *   Y[r][j]          = (a + W2 c) + (W1 b + W3 d)
 *   Y[r][j + L/4]    = (a - W2 c) - j (W1 b - W3 d)
 *   Y[r][j + L/2]    = (a + W2 c) - (W1 b + W3 d)
 *   Y[r][j + 3L/4]   = (a - W2 c) + j (W1 b - W3 d).
 * Each twiddle W^k (k < 3N/4) has its own table entry (m, t, path) from the
 * rules of Algorithm 1.  With the sine-path s1 negated, both paths write
 * W b = m * h, h = (h1, h2):
 *   cosine: h1 = s1 = b_r - t b_i, h2 = s2 = t b_r + b_i   (eq. (berg-s))
 *   sine:   h1 = -s1 = -(b_i - t b_r), h2 = s2 = b_r + t b_i (eq. (lf-s))
 * (two FMAs; negation is exact).  The odd pair W1 b +- W3 d = m1 h_b +- m3 h_d
 * takes the larger of |m1|, |m3| as its outer multiplier M and the ratio
 * rho = (smaller m) / (larger m), so |rho| <= 1 as every twiddle ratio:
 *   |m1| >= |m3|: M = m1, rho = m3/m1, g0 = h_b + rho h_d, g1 = h_b - rho h_d
 *   otherwise:    M = m3, rho = m1/m3, g0 = rho h_b + h_d, g1 = rho h_b - h_d
 * so that W1 b + W3 d = M g0 and W1 b - W3 d = M g1.  The butterfly is then
 *   h_b, h_c, h_d                       6 FMAs
 *   u0 = a + m2 h_c, u1 = a - m2 h_c    4 FMAs
 *   g0, g1                              4 FMAs
 *   Y0 = u0 + M g0, Y2 = u0 - M g0,
 *   Y1 = u1 - j M g1 = (u1_r + M g1_i, u1_i - M g1_r),
 *   Y3 = u1 + j M g1 = (u1_r - M g1_i, u1_i + M g1_r)   8 FMAs
 * 22 FMAs per radix-4 butterfly (two radix-2 stages take 24), each rounded
 * once.  rho and the choice of M come from the FP64 multipliers and rho is
 * rounded once to the working precision, like m and t.
 * The inverse transform (twiddles W^{-k}) turns the rotations -j and +j of
 * the odd terms into +j and -j: Y1 and Y3 trade places.
 */

/* Table of the radix-4 form: entries k < count of W^k for size n. */
int orc_table_count(int64_t n, int kind, int inverse, int64_t count, double* mult, double* ratio,
                    int32_t* path) {
    if (!is_pow2(n) || kind < 0 || kind > 3 || count < 0 || count > n) return -1;
    for (int64_t k = 0; k < count; ++k) table_entry(k, n, kind, inverse, &mult[k], &ratio[k], &path[k]);
    return 0;
}

/* Pair choice of the radix-4 butterfly for column j < n/4 of the last stage
 * (span n): sel = 1 when |m(W^j)| >= |m(W^{3j})| (outer multiplier m1), and
 * rho, both from the FP64 multipliers. */
static void pair_choice(double m1, double m3, int* sel, double* rho) {
    *sel = fabs(m1) >= fabs(m3);
    *rho = *sel ? m3 / m1 : m1 / m3;
}

int orc_pairs4(int64_t n, int kind, int inverse, double* rho, int32_t* sel) {
    if (!is_pow2(n) || n < 4 || kind < 0 || kind > 3) return -1;
    for (int64_t j = 0; j < n / 4; ++j) {
        double m1, t1, m3, t3;
        int32_t p1, p3;
        int s;
        table_entry(j, n, kind, inverse, &m1, &t1, &p1);
        table_entry(3 * j, n, kind, inverse, &m3, &t3, &p3);
        pair_choice(m1, m3, &s, &rho[j]);
        sel[j] = s;
    }
    return 0;
}

/* h = (h1, h2) with W b = m h (see above). */
static inline void scaled4(int prec, int path, double t, double br, double bi, double* h1, double* h2) {
    if (path == P_COS) {
        *h1 = fma_p(prec, -t, bi, br);
        *h2 = fma_p(prec, t, br, bi);
    } else {
        *h1 = -fma_p(prec, -t, br, bi);
        *h2 = fma_p(prec, t, bi, br);
    }
}

typedef struct { double m, t; int32_t path; } tw4_t;

static void bfly22(int prec, tw4_t w1, tw4_t w2, tw4_t w3, int sel, double rho,
                   const double* a, const double* b, const double* c, const double* d,
                   double* y0, double* y1, double* y2, double* y3) {
    double hb[2], hc[2], hd[2], u0[2], u1[2], g0[2], g1[2], M;
    scaled4(prec, w1.path, w1.t, b[0], b[1], &hb[0], &hb[1]);
    scaled4(prec, w2.path, w2.t, c[0], c[1], &hc[0], &hc[1]);
    scaled4(prec, w3.path, w3.t, d[0], d[1], &hd[0], &hd[1]);
    for (int i = 0; i < 2; ++i) {
        u0[i] = fma_p(prec, w2.m, hc[i], a[i]);
        u1[i] = fma_p(prec, -w2.m, hc[i], a[i]);
    }
    if (sel) {
        M = w1.m;
        for (int i = 0; i < 2; ++i) {
            g0[i] = fma_p(prec, rho, hd[i], hb[i]);
            g1[i] = fma_p(prec, ORC_MUTANT == 7 ? rho : -rho, hd[i], hb[i]);
        }
    } else {
        M = w3.m;
        for (int i = 0; i < 2; ++i) {
            g0[i] = fma_p(prec, rho, hb[i], hd[i]);
            g1[i] = fma_p(prec, rho, hb[i], -hd[i]);
        }
    }
    y0[0] = fma_p(prec, M, g0[0], u0[0]);
    y0[1] = fma_p(prec, M, g0[1], u0[1]);
    y2[0] = fma_p(prec, -M, g0[0], u0[0]);
    y2[1] = fma_p(prec, -M, g0[1], u0[1]);
    y1[0] = fma_p(prec, M, g1[1], u1[0]);
    y1[1] = fma_p(prec, ORC_MUTANT == 8 ? M : -M, g1[0], u1[1]);
    y3[0] = fma_p(prec, -M, g1[1], u1[0]);
    y3[1] = fma_p(prec, M, g1[0], u1[1]);
}

/* Canonical radix-4 order (see above) over the rounded table of W^k,
 * k < 3n/4 (mult, ratio, path) and the FP64 multipliers m64 for the pair
 * choice.  y, z: work arrays of 2n doubles; result left in y. */
static void stockham4_emulate(int64_t n, int prec, int inverse, const double* mult, const double* ratio,
                              const int32_t* path, const double* m64, double* y, double* z) {
    int mlog = log2i(n);
    int64_t L = 4;
    if (mlog % 2) {
        /* radix-2 stage of span 2: Y[r][0] = x[r] + x[r + n/2], Y[r][1] = difference */
        for (int64_t r = 0; r < n / 2; ++r) {
            double Ar, Ai, Br, Bi;
            bfly6(prec, path[0], mult[0], ratio[0], y[2 * r], y[2 * r + 1], y[2 * (r + n / 2)],
                  y[2 * (r + n / 2) + 1], &Ar, &Ai, &Br, &Bi);
            z[2 * r] = Ar; z[2 * r + 1] = Ai;
            z[2 * (r + n / 2)] = Br; z[2 * (r + n / 2) + 1] = Bi;
        }
        memcpy(y, z, sizeof(double) * 2 * (size_t)n);
        L = 8;
    }
    for (; L <= n; L *= 4) {
        int64_t nl = n / L, q4 = L / 4;
        for (int64_t r = 0; r < nl; ++r) {
            for (int64_t j = 0; j < q4; ++j) {
                int64_t k1 = j * nl, k2 = 2 * k1, k3 = 3 * k1;
                tw4_t w1 = {mult[k1], ratio[k1], path[k1]};
                tw4_t w2 = {mult[k2], ratio[k2], path[k2]};
                tw4_t w3 = {mult[k3], ratio[k3], path[k3]};
                int sel;
                double rho;
                pair_choice(m64[k1], m64[k3], &sel, &rho);
                if (ORC_MUTANT != 9) rho = round_p(prec, rho);
                const double* a = y + 2 * (r + 4 * nl * j);
                const double* b = y + 2 * (r + nl + 4 * nl * j);
                const double* c = y + 2 * (r + 2 * nl + 4 * nl * j);
                const double* d = y + 2 * (r + 3 * nl + 4 * nl * j);
                int64_t p1 = inverse ? 3 : 1, p3 = inverse ? 1 : 3;
                bfly22(prec, w1, w2, w3, sel, rho, a, b, c, d, z + 2 * (r + nl * j),
                       z + 2 * (r + nl * (j + p1 * q4)), z + 2 * (r + nl * (j + 2 * q4)),
                       z + 2 * (r + nl * (j + p3 * q4)));
            }
        }
        memcpy(y, z, sizeof(double) * 2 * (size_t)n);
    }
}

static int emulate4_batch(int64_t n, int64_t batch, int kind, int inverse, int prec,
                          const double* in, double* out) {
    if (!is_pow2(n) || batch < 0 || kind < 0 || kind > 3) return -1;
    int64_t cnt = n < 4 ? 1 : 3 * n / 4;
    double* mult = (double*)malloc(sizeof(double) * cnt);
    double* ratio = (double*)malloc(sizeof(double) * cnt);
    double* m64 = (double*)malloc(sizeof(double) * cnt);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * cnt);
    if (!mult || !ratio || !m64 || !path) {
        free(mult); free(ratio); free(m64); free(path);
        return -1;
    }
    orc_table_count(n, kind, inverse, cnt, mult, ratio, path);
    for (int64_t k = 0; k < cnt; ++k) {
        m64[k] = mult[k];
        mult[k] = round_p(prec, mult[k]);
        ratio[k] = round_p(prec, ratio[k]);
    }
    int err = 0;
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        if (!y || !z) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(static)
        for (int64_t b = 0; b < batch; ++b) {
            if (!y || !z) continue;
            for (int64_t i = 0; i < 2 * n; ++i) y[i] = round_p(prec, in[b * 2 * n + i]);
            stockham4_emulate(n, prec, inverse, mult, ratio, path, m64, y, z);
            memcpy(out + b * 2 * n, y, sizeof(double) * 2 * (size_t)n);
        }
        free(y); free(z);
    }
    free(mult); free(ratio); free(m64); free(path);
    return err;
}

int orc_emulate4_f64(int64_t n, int64_t batch, int kind, int inverse, const double* in, double* out) {
    return emulate4_batch(n, batch, kind, inverse, PREC_F64, in, out);
}

int orc_emulate4_f32(int64_t n, int64_t batch, int kind, int inverse, const float* in, float* out) {
    size_t cnt = (size_t)(2 * n * batch);
    double* a = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    double* b = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    if (!a || !b) { free(a); free(b); return -1; }
    for (size_t i = 0; i < cnt; ++i) a[i] = (double)in[i];
    int rc = emulate4_batch(n, batch, kind, inverse, PREC_F32, a, b);
    for (size_t i = 0; i < cnt && rc == 0; ++i) out[i] = (float)b[i];
    free(a); free(b);
    return rc;
}

int orc_emulate4_f16(int64_t n, int64_t batch, int kind, int inverse, const uint16_t* in, uint16_t* out) {
    size_t cnt = (size_t)(2 * n * batch);
    double* a = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    double* b = (double*)malloc(sizeof(double) * (cnt ? cnt : 1));
    if (!a || !b) { free(a); free(b); return -1; }
    for (size_t i = 0; i < cnt; ++i) a[i] = orc_f16_to_double(in[i]);
    int rc = emulate4_batch(n, batch, kind, inverse, PREC_F16, a, b);
    for (size_t i = 0; i < cnt && rc == 0; ++i) out[i] = orc_rn16(b[i]);
    free(a); free(b);
    return rc;
}

/* ------------------------------------------------------------ FP64 reference */

/*
 * Plain radix-2 Stockham FFT in FP64 with the 10-flop butterfly of
 * eqs. (std1)-(std2): A = a + (w_r b_r - w_i b_i, w_i b_r + w_r b_i), B = a - (...).
 */
int orc_fft64(int64_t n, int64_t batch, int inverse, const double* in, double* out) {
    if (!is_pow2(n) || batch < 0) return -1;
    int64_t h2 = n / 2;
    double* wr = (double*)malloc(sizeof(double) * h2);
    double* wi = (double*)malloc(sizeof(double) * h2);
    if (!wr || !wi) { free(wr); free(wi); return -1; }
    for (int64_t k = 0; k < h2; ++k) {
        double th = orc_theta(k, n);
        wr[k] = cos(th);
        wi[k] = inverse ? -sin(th) : sin(th);
    }
    int mlog = log2i(n);
    int err = 0;
#pragma omp parallel
    {
        double* y = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        if (!y || !z) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(static)
        for (int64_t b = 0; b < batch; ++b) {
            if (!y || !z) continue;
            memcpy(y, in + b * 2 * n, sizeof(double) * 2 * (size_t)n);
            for (int s = 1; s <= mlog; ++s) {
                int64_t L = (int64_t)1 << s, h = L / 2, nl = n / L, nh = n / h;
                for (int64_t r = 0; r < nl; ++r) {
                    for (int64_t j = 0; j < h; ++j) {
                        int64_t k = j * nl;
                        int64_t ia = r + nh * j, ib = r + nl + nh * j;
                        int64_t oa = r + nl * j, ob = r + nl * (j + h);
                        double br = y[2 * ib], bi = y[2 * ib + 1];
                        double pr = wr[k] * br - wi[k] * bi;
                        double pi = wi[k] * br + wr[k] * bi;
                        z[2 * oa] = y[2 * ia] + pr;
                        z[2 * oa + 1] = y[2 * ia + 1] + pi;
                        z[2 * ob] = y[2 * ia] - pr;
                        z[2 * ob + 1] = y[2 * ia + 1] - pi;
                    }
                }
                memcpy(y, z, sizeof(double) * 2 * (size_t)n);
            }
            memcpy(out + b * 2 * n, y, sizeof(double) * 2 * (size_t)n);
        }
        free(y); free(z);
    }
    free(wr); free(wi);
    return err;
}

/* The DFT of eq. (1) written out: X[k] = sum_n x[n] exp(-j 2 pi (n k mod N) / N);
 * inverse != 0: exp(+j 2 pi (n k mod N) / N). */
int orc_dft64(int64_t n, int64_t batch, int inverse, const double* in, double* out) {
    if (n < 1 || batch < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; ++b) {
        const double* x = in + b * 2 * n;
        double* X = out + b * 2 * n;
        for (int64_t k = 0; k < n; ++k) {
            double sr = 0.0, si = 0.0;
            for (int64_t t = 0; t < n; ++t) {
                double th = orc_theta((t * k) % n, n);
                double c = cos(th), s = inverse ? -sin(th) : sin(th);
                sr += x[2 * t] * c - x[2 * t + 1] * s;
                si += x[2 * t] * s + x[2 * t + 1] * c;
            }
            X[2 * k] = sr;
            X[2 * k + 1] = si;
        }
    }
    return 0;
}
