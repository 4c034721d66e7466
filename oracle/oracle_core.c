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
int orc_table_dir(int64_t n, int kind, int inverse, double* mult, double* ratio, int32_t* path) {
    if (!is_pow2(n) || kind < 0 || kind > 3) return -1;
    for (int64_t k = 0; k < n / 2; ++k) {
        double th = orc_theta(k, n);
        double wr = cos(th), wi = sin(th);
        if (inverse) wi = -wi;                  /* W^{-k}: the conjugate */
        int use_cos;
        if (kind == K_DUAL_SELECT) use_cos = fabs(wr) >= fabs(wi);
        else if (kind == K_COSINE) use_cos = 1;
        else if (kind == K_LF_W0_EXEMPT) use_cos = (k == 0);
        else use_cos = 0;
        if (use_cos) {
            mult[k] = wr;
            ratio[k] = wi / wr;
            path[k] = P_COS;
        } else {
            double d = wi;
            if (kind == K_LINZER_FEIG && fabs(d) < ORC_EPS_CLAMP) d = ORC_EPS_CLAMP;
            mult[k] = d;
            ratio[k] = wr / d;
            path[k] = P_SIN;
        }
    }
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
