// Device side of the dual-select FFT for gfx950 (CDNA4, wave64).
//
// One kernel template covers three ways of cutting a batch of transforms into
// "units", each unit being a run of consecutive radix-2 Stockham stages done
// inside one workgroup:
//   MODE_SMALL  the whole transform is one unit (N fits one workgroup's LDS);
//   MODE_COLS   first kernel of the two-pass schedule: stages 1..log2(NU) of
//               the decimated column x[r0 + (N/NU) i], i < NU, per unit;
//   MODE_ROWS   second kernel: stages log2(N/NU)+1..log2(N) of row q0 of the
//               intermediate Y[i][q0], i < NU, per unit.
// Inside a unit, stages are fused into register passes of radix R = 2^LR; each
// lane holds E elements (E/R groups of R) and runs the pass's LR radix-2 stages
// in registers; passes exchange data through LDS.
//
// Every radix-2 butterfly is the six-FMA butterfly of the paper (arXiv
// 2604.00567): eqs. (berg-s)-(berg-B) on the cosine path, eqs. (lf-s)-(lf-B)
// on the sine path, with the same operands, twiddle and FMA association as the
// radix-2 Stockham definition, so fusing stages changes no rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace dsfft {

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));

// Device twiddle entry, binary16 plan.  w = (sigma*m, m) as two halves (low =
// sigma*m), sigma = +1 on the cosine path and -1 on the sine path; ts carries
// the path as a rotate amount in its low 16 bits (0 cosine, 16 sine) and the
// ratio t as a binary16 value in its high 16 bits.
struct TwH {
    uint32_t w;
    uint32_t ts;
};

// Device twiddle entry, binary32 plan: (sigma*m, m, t) and a lane mask that is
// all ones on the sine path.
struct __attribute__((aligned(16))) TwF {
    float sm;
    float m;
    float t;
    uint32_t mask;
};

__device__ __forceinline__ h2_t as_h2(uint32_t u) { return __builtin_bit_cast(h2_t, u); }
__device__ __forceinline__ uint32_t as_u32(h2_t h) { return __builtin_bit_cast(uint32_t, h); }

// Six-FMA butterfly, binary16 (three packed v_pk_fma_f16 = six FMAs).
//   c = b on the cosine path, (b_i, b_r) on the sine path (one v_alignbit);
//   (s1, s2) = (c.lo - t c.hi, t c.lo + c.hi)
//     cosine: (b_r - t b_i, t b_r + b_i)             eq. (berg-s)
//     sine:   (b_i - t b_r, t b_i + b_r)             eq. (lf-s), s2 read as b_r + t b_i
//   A = a + (s1, s2) * (sigma m, m),  B = a - (s1, s2) * (sigma m, m)
//     cosine: A_r = a_r + s1 m, A_i = a_i + s2 m     eqs. (berg-A), (berg-B)
//     sine:   A_r = a_r - s1 m, A_i = a_i + s2 m     eqs. (lf-A), (lf-B)
// Negating an operand is exact, so each lane computes the same FMAs as the
// printed equations.
__device__ __forceinline__ void bfly(uint32_t& a, uint32_t& b, const TwH tw) {
    const uint32_t c = __builtin_amdgcn_alignbit(b, b, tw.ts);
    const h2_t cv = as_h2(c);
    const h2_t tv = as_h2(tw.ts);
    const h2_t w = as_h2(tw.w);
    const h2_t av = as_h2(a);
    h2_t tt;
    tt.x = -tv.y;
    tt.y = tv.y;
    const h2_t s = __builtin_elementwise_fma(tt, cv.yx, cv);
    const h2_t A = __builtin_elementwise_fma(s, w, av);
    const h2_t B = __builtin_elementwise_fma(-s, w, av);
    a = as_u32(A);
    b = as_u32(B);
}

// Six-FMA butterfly, binary32 (six v_fma_f32); the path picks (c_r, c_i) from
// (b_r, b_i) or (b_i, b_r) with a bitwise select on the table's lane mask.
// (The vector elements are copied to scalars before the bit casts: clang's
// __builtin_bit_cast applied directly to an ext_vector element reads element 0.)
__device__ __forceinline__ void bfly(f2_t& a, f2_t& b, const TwF tw) {
    const float bxf = b.x, byf = b.y;
    const uint32_t br = __builtin_bit_cast(uint32_t, bxf);
    const uint32_t bi = __builtin_bit_cast(uint32_t, byf);
    const float cr = __builtin_bit_cast(float, (tw.mask & bi) | (~tw.mask & br));
    const float ci = __builtin_bit_cast(float, (tw.mask & br) | (~tw.mask & bi));
    const float s1 = __builtin_fmaf(-tw.t, ci, cr);
    const float s2 = __builtin_fmaf(tw.t, cr, ci);
    f2_t A, B;
    A.x = __builtin_fmaf(s1, tw.sm, a.x);
    A.y = __builtin_fmaf(s2, tw.m, a.y);
    B.x = __builtin_fmaf(-s1, tw.sm, a.x);
    B.y = __builtin_fmaf(-s2, tw.m, a.y);
    a = A;
    b = B;
}

// The same binary32 butterfly on operands still held as stored binary16 pairs
// (the first stage of a binary16-storage plan): the path's operand order is a
// rotate of the packed pair by 16 bits, and each widening, which is exact,
// folds into its FMA (v_fma_mix_f32), so the FMAs, their operands and their
// roundings are those of widening first and calling bfly.
__device__ __forceinline__ void bfly_stored(uint32_t a, uint32_t b, const TwF tw, f2_t& A, f2_t& B) {
    const uint32_t c = __builtin_amdgcn_alignbit(b, b, tw.mask & 16u);
    const float cr = (float)__builtin_bit_cast(_Float16, (uint16_t)c);
    const float ci = (float)__builtin_bit_cast(_Float16, (uint16_t)(c >> 16));
    const float ar = (float)__builtin_bit_cast(_Float16, (uint16_t)a);
    const float ai = (float)__builtin_bit_cast(_Float16, (uint16_t)(a >> 16));
    const float s1 = __builtin_fmaf(-tw.t, ci, cr);
    const float s2 = __builtin_fmaf(tw.t, cr, ci);
    A.x = __builtin_fmaf(s1, tw.sm, ar);
    A.y = __builtin_fmaf(s2, tw.m, ai);
    B.x = __builtin_fmaf(-s1, tw.sm, ar);
    B.y = __builtin_fmaf(-s2, tw.m, ai);
}

// Encodings of the path choice (the select flag of Sec. III; Sec. VI notes
// that the branch on it can become an operand order held in the table):
//   ENC_TABLE   the table entry carries the operand order (a rotate amount)
//               and the multiplier with the path's sign (sigma m, m): no
//               branch, no select (the form every kernel uses by default);
//   ENC_SELECT  each lane selects the operand order and the multiplier's
//               sign from the path flag (v_cndmask);
//   ENC_BRANCH  each lane branches on the path flag and runs that path's
//               code (lanes of one wave on both paths run both).
// All three compute the same FMAs on the same operands (bit-identical);
// binary16 kernels only (the binary32 butterfly always uses a lane mask).
//   ENC_RADIX4  not a path encoding: the radix-4 form of the method (Sec. VI,
//               generality), whose butterflies combine four inputs with 22
//               FMAs and read radix-4 table entries (Tw4H / Tw4F); a
//               different canonical order, so results differ from radix 2.
enum { ENC_TABLE = 0, ENC_SELECT = 1, ENC_BRANCH = 2, ENC_RADIX4 = 3 };

template <int ENC>
__device__ __forceinline__ void bfly_enc(uint32_t& a, uint32_t& b, const TwH tw) {
    if constexpr (ENC == ENC_TABLE) {
        bfly(a, b, tw);
    } else {
        const bool sine = (tw.ts & 16u) != 0;      // the path flag
        const h2_t tv = as_h2(tw.ts);
        const _Float16 m = as_h2(tw.w).y;           // the multiplier, unsigned by path
        const h2_t av = as_h2(a);
        h2_t tt;
        tt.x = -tv.y;
        tt.y = tv.y;
        h2_t A, B;
        if constexpr (ENC == ENC_SELECT) {
            const uint32_t c = sine ? __builtin_amdgcn_alignbit(b, b, 16) : b;
            h2_t w;
            w.x = sine ? -m : m;
            w.y = m;
            const h2_t cv = as_h2(c);
            const h2_t s = __builtin_elementwise_fma(tt, cv.yx, cv);
            A = __builtin_elementwise_fma(s, w, av);
            B = __builtin_elementwise_fma(-s, w, av);
        } else if (sine) {
            asm volatile("");                        // keeps the branch (no if-conversion)
            const h2_t cv = as_h2(__builtin_amdgcn_alignbit(b, b, 16));   // (b_i, b_r)
            h2_t w;
            w.x = -m;
            w.y = m;
            const h2_t s = __builtin_elementwise_fma(tt, cv.yx, cv);
            A = __builtin_elementwise_fma(s, w, av);
            B = __builtin_elementwise_fma(-s, w, av);
        } else {
            asm volatile("");
            const h2_t bv = as_h2(b);
            h2_t w;
            w.x = m;
            w.y = m;
            const h2_t s = __builtin_elementwise_fma(tt, bv.yx, bv);
            A = __builtin_elementwise_fma(s, w, av);
            B = __builtin_elementwise_fma(-s, w, av);
        }
        a = as_u32(A);
        b = as_u32(B);
    }
}
template <int ENC>
__device__ __forceinline__ void bfly_enc(f2_t& a, f2_t& b, const TwF tw) {
    bfly(a, b, tw);
}

template <class E> struct TwOf;
template <> struct TwOf<uint32_t> { using type = TwH; };
template <> struct TwOf<f2_t> { using type = TwF; };

// ------------------------------------------------------- radix-4 butterflies
//
// Radix-4 form of the method (Sec. VI: in a higher-radix butterfly each
// twiddle multiplication picks its own bounded-ratio factorisation).  A
// radix-4 stage of span L combines, for column j < L/4, the four span-L/4
// DFTs a, b, c, d at residues r + p N/L with W1 = W_L^j, W2 = W1^2, W3 = W1^3:
//   Y0 = (a + W2 c) + (W1 b + W3 d),   Y2 = (a + W2 c) - (W1 b + W3 d),
//   Y1 = (a - W2 c) - j (W1 b - W3 d), Y3 = (a - W2 c) + j (W1 b - W3 d)
// (Y_p at column j + p L/4).  Each W^k of the three takes its own table entry
// (m_k, t_k, path_k) by the rules of Algorithm 1, and W^k x = m_k h_k(x) with
//   h = (x_r - t x_i, t x_r + x_i)        cosine path (eq. (berg-s))
//   h = (-(x_i - t x_r), x_r + t x_i)     sine path (eq. (lf-s), s1 negated).
// The odd pair W1 b +- W3 d = m1 h_b +- m3 h_d takes the larger of |m1|, |m3|
// as outer multiplier M and rho = smaller/larger (|rho| <= 1, like every
// ratio):  |m1| >= |m3|: g0 = h_b + rho h_d, g1 = h_b - rho h_d (M = m1);
//          otherwise:    g0 = rho h_b + h_d, g1 = rho h_b - h_d (M = m3).
// Then u0 = a + m2 h_c, u1 = a - m2 h_c, Y0/Y2 = u0 +- M g0,
// Y1 = (u1_r + M g1_i, u1_i - M g1_r), Y3 = (u1_r - M g1_i, u1_i + M g1_r):
// 22 FMAs, each rounded once (two radix-2 stages take 24).
//
// Device form.  With s_x = (x.lo - t x.hi, t x.lo + x.hi) of the path-ordered
// operand (as in the radix-2 butterfly) h = (sigma s.lo, s.hi), sigma = -1 on
// the sine path.  Negation is exact (RN(-v) = -RN(v)), so every sign folds
// into the table's multipliers: with (x, y) = (s_d, s_b) when M = m1 and
// (s_b, s_d) otherwise,
//   g0' = y + (sigma1 sigma3 rho, rho) x,   g1'' = y - (sigma1 sigma3 rho, rho) x,
//   g0 = D g0',  g1 = sg D g1''   (D = diag(sigma_M, 1), sg = +1 when M = m1, -1 otherwise),
//   Y0 = u0 + (sigma_M M, M) g0',  Y2 = u0 - (sigma_M M, M) g0',
//   Y1 = u1 + (sg M, -sg sigma_M M) g1''.yx,  Y3 = u1 - (sg M, -sg sigma_M M) g1''.yx,
// which are the same FMAs on the same operands as the definition.  The
// inverse transform (conjugate twiddles) swaps the places of Y1 and Y3; the
// inverse table stores the last multiplier negated, which makes that swap.
//
// Radix-4 table: entry L/4 + j holds the butterfly of span L, column j
// (L = 4, 8, 16, ...: every level fits in [1, N_cap/2)); entry 0 holds the
// radix-2 butterfly of W^0 in (ts1, w2), for the span-2 stage that comes first
// when log2 N is odd.
struct __attribute__((aligned(16))) Tw4H {
    uint32_t ts1, ts2, ts3;   // operand order | ratio << 16 of W1, W2, W3 (as TwH::ts)
    uint32_t w2;              // (sigma2 m2, m2)
    uint32_t rr;              // (sigma1 sigma3 rho, rho)
    uint32_t mm0;             // (sigma_M M, M)
    uint32_t mm1;             // (sg M, -sg sigma_M M), negated in the inverse table
    uint32_t msel;            // all ones when M = m1
};
struct __attribute__((aligned(16))) Tw4F {
    float t1, t2, t3;
    uint32_t mask1, mask2, mask3;   // all ones on the sine path (as TwF::mask)
    float sm2, m2;
    float srho, rho;
    float smM, M;
    float mma, mmb;
    uint32_t msel, pad;
};

// s = (c.lo - t c.hi, t c.lo + c.hi) of the path-ordered operand c.
__device__ __forceinline__ h2_t scaled_pair(uint32_t b, uint32_t ts) {
    const h2_t cv = as_h2(__builtin_amdgcn_alignbit(b, b, ts));
    const h2_t tv = as_h2(ts);
    h2_t tt;
    tt.x = -tv.y;
    tt.y = tv.y;
    return __builtin_elementwise_fma(tt, cv.yx, cv);
}
__device__ __forceinline__ f2_t scaled_pair(f2_t b, float t, uint32_t mask) {
    const float bxf = b.x, byf = b.y;
    const uint32_t br = __builtin_bit_cast(uint32_t, bxf);
    const uint32_t bi = __builtin_bit_cast(uint32_t, byf);
    const float cr = __builtin_bit_cast(float, (mask & bi) | (~mask & br));
    const float ci = __builtin_bit_cast(float, (mask & br) | (~mask & bi));
    f2_t s;
    s.x = __builtin_fmaf(-t, ci, cr);
    s.y = __builtin_fmaf(t, cr, ci);
    return s;
}
__device__ __forceinline__ uint32_t bitsel(uint32_t m, uint32_t x, uint32_t y) { return (m & x) | (~m & y); }

// Radix-4 butterfly, binary16: 11 packed FMAs (22 FMAs); (a, b, c, d) -> (Y0, Y1, Y2, Y3).
__device__ __forceinline__ void bfly4(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d, const Tw4H& w) {
    const h2_t sb = scaled_pair(b, w.ts1);
    const h2_t sc = scaled_pair(c, w.ts2);
    const h2_t sd = scaled_pair(d, w.ts3);
    const h2_t av = as_h2(a);
    const h2_t w2 = as_h2(w.w2);
    const h2_t u0 = __builtin_elementwise_fma(sc, w2, av);
    const h2_t u1 = __builtin_elementwise_fma(-sc, w2, av);
    const h2_t x = as_h2(bitsel(w.msel, as_u32(sd), as_u32(sb)));
    const h2_t y = as_h2(bitsel(w.msel, as_u32(sb), as_u32(sd)));
    const h2_t rr = as_h2(w.rr);
    const h2_t g0 = __builtin_elementwise_fma(x, rr, y);
    const h2_t g1 = __builtin_elementwise_fma(-x, rr, y);
    const h2_t mm0 = as_h2(w.mm0), mm1 = as_h2(w.mm1);
    a = as_u32(__builtin_elementwise_fma(g0, mm0, u0));
    c = as_u32(__builtin_elementwise_fma(-g0, mm0, u0));
    b = as_u32(__builtin_elementwise_fma(g1.yx, mm1, u1));
    d = as_u32(__builtin_elementwise_fma(-g1.yx, mm1, u1));
}

// Radix-4 butterfly, binary32: 22 v_fma_f32.
__device__ __forceinline__ void bfly4(f2_t& a, f2_t& b, f2_t& c, f2_t& d, const Tw4F& w) {
    const f2_t sb = scaled_pair(b, w.t1, w.mask1);
    const f2_t sc = scaled_pair(c, w.t2, w.mask2);
    const f2_t sd = scaled_pair(d, w.t3, w.mask3);
    const float ax = a.x, ay = a.y;
    const float u0x = __builtin_fmaf(sc.x, w.sm2, ax), u0y = __builtin_fmaf(sc.y, w.m2, ay);
    const float u1x = __builtin_fmaf(-sc.x, w.sm2, ax), u1y = __builtin_fmaf(-sc.y, w.m2, ay);
    const float sbx = sb.x, sby = sb.y, sdx = sd.x, sdy = sd.y;
    const uint32_t bx = __builtin_bit_cast(uint32_t, sbx), by = __builtin_bit_cast(uint32_t, sby);
    const uint32_t dx = __builtin_bit_cast(uint32_t, sdx), dy = __builtin_bit_cast(uint32_t, sdy);
    const float xx = __builtin_bit_cast(float, bitsel(w.msel, dx, bx));
    const float xy = __builtin_bit_cast(float, bitsel(w.msel, dy, by));
    const float yx = __builtin_bit_cast(float, bitsel(w.msel, bx, dx));
    const float yy = __builtin_bit_cast(float, bitsel(w.msel, by, dy));
    const float g0x = __builtin_fmaf(xx, w.srho, yx), g0y = __builtin_fmaf(xy, w.rho, yy);
    const float g1x = __builtin_fmaf(-xx, w.srho, yx), g1y = __builtin_fmaf(-xy, w.rho, yy);
    f2_t y0, y1, y2, y3;
    y0.x = __builtin_fmaf(g0x, w.smM, u0x);
    y0.y = __builtin_fmaf(g0y, w.M, u0y);
    y2.x = __builtin_fmaf(-g0x, w.smM, u0x);
    y2.y = __builtin_fmaf(-g0y, w.M, u0y);
    y1.x = __builtin_fmaf(g1y, w.mma, u1x);
    y1.y = __builtin_fmaf(g1x, w.mmb, u1y);
    y3.x = __builtin_fmaf(-g1y, w.mma, u1x);
    y3.y = __builtin_fmaf(-g1x, w.mmb, u1y);
    a = y0;
    b = y1;
    c = y2;
    d = y3;
}

// The radix-2 butterfly of the span-2 stage (odd log2 N) from entry 0.
__device__ __forceinline__ void bfly_w0(uint32_t& a, uint32_t& b, const Tw4H& w) { bfly(a, b, TwH{w.w2, w.ts1}); }
__device__ __forceinline__ void bfly_w0(f2_t& a, f2_t& b, const Tw4F& w) {
    bfly(a, b, TwF{w.sm2, w.m2, w.t1, w.mask1});
}

// Table entry type of a kernel: radix-2 entries, or radix-4 ones (ENC_RADIX4).
template <class E, int ENC> struct TwOfEnc { using type = typename TwOf<E>::type; };
template <> struct TwOfEnc<uint32_t, ENC_RADIX4> { using type = Tw4H; };
template <> struct TwOfEnc<f2_t, ENC_RADIX4> { using type = Tw4F; };
template <class E, int ENC> using TwT = typename TwOfEnc<E, ENC>::type;

// Storage and compute types.  A kernel computes in E; its input and output
// may be stored in another type S (binary16 storage with binary32
// butterflies: S = binary16 pair, E = binary32 pair).  Loads widen exactly,
// stores round once, to nearest even; with S = E both are the identity.
__device__ __forceinline__ uint32_t to_storage(uint32_t v, uint32_t) { return v; }
__device__ __forceinline__ f2_t to_storage(f2_t v, f2_t) { return v; }
// One v_cvt_f16_f32 per half (rounding by the mode register: to nearest
// even).  The compiler would otherwise pair the two halves into
// v_cvt_pk_f16_f32, which on gfx950 resolved exact ties to the odd
// neighbour in testing, not to the even one.
__device__ __forceinline__ uint32_t to_storage(f2_t v, uint32_t) {
    const float x = v.x, y = v.y;
    uint32_t lo, hi;
    asm("v_cvt_f16_f32 %0, %1" : "=v"(lo) : "v"(x));
    asm("v_cvt_f16_f32 %0, %1" : "=v"(hi) : "v"(y));
    return (lo & 0xffffu) | (hi << 16);
}
__device__ __forceinline__ uint32_t to_compute(uint32_t s, uint32_t) { return s; }
__device__ __forceinline__ f2_t to_compute(f2_t s, f2_t) { return s; }
__device__ __forceinline__ f2_t to_compute(uint32_t s, f2_t) {
    const h2_t h = as_h2(s);
    f2_t v;
    v.x = (float)h.x;
    v.y = (float)h.y;
    return v;
}
// STREAM: the streaming (non-temporal) hint; a compile-time choice, so that
// each access is emitted in exactly one form.
template <bool STREAM, class E, class S>
__device__ __forceinline__ E load_elem(const S* p) {
    if constexpr (STREAM) return to_compute(__builtin_nontemporal_load(p), E{});
    else return to_compute(*p, E{});
}
template <bool STREAM, class E, class S>
__device__ __forceinline__ void store_elem(E v, S* p) {
    const S s = to_storage(v, S{});
    if constexpr (STREAM) __builtin_nontemporal_store(s, p);
    else *p = s;
}

// Whole-transform blocks (a workgroup's units contiguous in memory) of units
// larger than 4 KiB move through a buffer resource over the block (smaller
// units address every element with the global instructions' immediate
// offset, and their one-transform-per-lane patterns measured several times
// slower through buffer instructions): each access is the lane's 32-bit
// byte offset plus a compile-time offset held in a scalar register, so no
// per-access 64-bit address arithmetic runs on the vector ALU (which the
// largest transforms, at 6 FMAs per byte, cannot spare), and accesses past
// the block's end read zero and write nothing.  Word 3 of a gfx9 buffer
// descriptor for raw (unformatted) dword access is 0x00020000.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
template <class S>
__device__ __forceinline__ rsrc_t block_rsrc(const S* base, int64_t elems) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base), 0, (int)(elems * (int64_t)sizeof(S)),
                                             0x00020000);
}
// Cache policy: 2 = non-temporal (streaming), as __builtin_nontemporal_load/store.
// A constant offset below 4096 fits the instruction's own offset field; larger
// ones go to the scalar offset register.
template <bool STREAM, class E, class S>
__device__ __forceinline__ E buf_load(rsrc_t r, uint32_t lane_off, uint32_t c) {
    const uint32_t voff = c < 4096 ? lane_off + c : lane_off;
    const uint32_t soff = c < 4096 ? 0 : c;
    if constexpr (sizeof(S) == 4) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, STREAM ? 2 : 0);
        return to_compute(__builtin_bit_cast(S, u), E{});
    } else {
        static_assert(sizeof(S) == 8, "binary16 or binary32 pairs");
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, STREAM ? 2 : 0);
        return to_compute(__builtin_bit_cast(S, u), E{});
    }
}
template <bool STREAM, class E, class S>
__device__ __forceinline__ void buf_store(E v, rsrc_t r, uint32_t lane_off, uint32_t c) {
    const uint32_t voff = c < 4096 ? lane_off + c : lane_off;
    const uint32_t soff = c < 4096 ? 0 : c;
    const S s = to_storage(v, S{});
    if constexpr (sizeof(S) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, s), r, voff, soff, STREAM ? 2 : 0);
    } else {
        typedef uint32_t u2_t __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, s), r, voff, soff, STREAM ? 2 : 0);
    }
}

// Level-ordered twiddle table: entry L/2 + j is T_L[j] = W_L^j for span L (a
// power of two) and j < L/2, stored as TwH/TwF.  Since theta = -(2 pi j)/L
// scales exactly by powers of two, T_L[j] equals T_N[j N / L] bit for bit, so
// one table of capacity N_cap serves every N <= N_cap.  For a group whose
// butterflies have global column index j = qg + Lg0 * (2^(t-1) + e) in stage t
// of a radix-R pass, the twiddle is entry qg + Lg0 * c with c = 2^(t-1) + e in
// [1, R).

// Radix-R register pass on one group of R = 2^LR elements (v[0..R)).  Stage t
// (1..LR) pairs v[i + 2He] with v[i + H + 2He] (H = R >> t, i < H, e < 2^(t-1))
// under twiddle c = 2^(t-1) + e, and writes A to v[i + He], B to v[i + He + R/2].
// On entry v[i] = Y[r + M i][q]; on exit v[e] = Y'[r][q + L0 e].
// Radix-4 form: the same group layout, radix-4 stages (and, for the first pass
// of an odd log2 N, the span-2 radix-2 stage before them).  With S columns
// done (H = R / S residues left), v[i + H e] holds residue i, column e; a
// radix-4 stage takes a, b, c, d = v[i + H e + p H/4] (p < 4) under entry
// c = S + e and writes output p to v[i + (H/4) (e + p S)].
template <int LR, bool ODD, class E, class TW>
__device__ __forceinline__ void reg_pass4(E* v, const TW* tw) {
    constexpr int R = 1 << LR;
    static_assert((LR - (ODD ? 1 : 0)) % 2 == 0, "radix-4 stages fill the pass");
    if constexpr (ODD) {
        E nv[R];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            E a = v[i], b = v[i + R / 2];
            bfly_w0(a, b, tw[0]);
            nv[i] = a;
            nv[i + R / 2] = b;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = nv[k];
    }
#pragma unroll
    for (int S = ODD ? 2 : 1; S < R; S *= 4) {
        const int H = R / S, H4 = H / 4;
        E nv[R];
#pragma unroll
        for (int e = 0; e < S; ++e) {
#pragma unroll
            for (int i = 0; i < H4; ++i) {
                E a = v[i + H * e], b = v[i + H4 + H * e], c = v[i + 2 * H4 + H * e], d = v[i + 3 * H4 + H * e];
                bfly4(a, b, c, d, tw[S + e]);
                nv[i + H4 * e] = a;
                nv[i + H4 * (e + S)] = b;
                nv[i + H4 * (e + 2 * S)] = c;
                nv[i + H4 * (e + 3 * S)] = d;
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = nv[k];
    }
}

// T0 > 1: stages before T0 are done already (a binary16-storage first pass).
template <int LR, int ENC = ENC_TABLE, bool ODD = false, int T0 = 1, class E, class TW>
__device__ __forceinline__ void reg_pass(E* v, const TW* tw) {
    if constexpr (ENC == ENC_RADIX4) {
        static_assert(T0 == 1, "radix-4 passes start at their first stage");
        reg_pass4<LR, ODD>(v, tw);
    } else {
        constexpr int R = 1 << LR;
#pragma unroll
        for (int t = T0; t <= LR; ++t) {
            const int H = R >> t;
            E nv[R];
#pragma unroll
            for (int e = 0; e < (1 << (t - 1)); ++e) {
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    E a = v[i + 2 * H * e];
                    E b = v[i + H + 2 * H * e];
                    bfly_enc<ENC>(a, b, tw[(1 << (t - 1)) + e]);
                    nv[i + H * e] = a;
                    nv[i + H * e + R / 2] = b;
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) v[k] = nv[k];
        }
    }
}

enum { MODE_SMALL = 0, MODE_COLS = 1, MODE_ROWS = 2 };

// ------------------------------------------------------------ compile-time plan

template <int LOG_NU, int LR0, int LR1, int LR2, int LANE = 0>
struct PassPlan {
    static constexpr int log_nu = LOG_NU;
    static constexpr int NP = LR1 == 0 ? 1 : (LR2 == 0 ? 2 : 3);
    static constexpr int lr(int p) { return p == 0 ? LR0 : (p == 1 ? LR1 : LR2); }
    // log2 of the span before pass p
    static constexpr int log_l0(int p) { return p == 0 ? 0 : (p == 1 ? LR0 : LR0 + LR1); }
    // log2 of M after pass p: residues left = NU / (R_p L0_p)
    static constexpr int log_m(int p) { return LOG_NU - log_l0(p) - lr(p); }
    // LDS padding for the exchange after pass p: PAD elements per row of M_p
    // elements, PAD = M_{p+1} (residues left after the next pass) when that is
    // below 32, which spreads group-fast reads of consecutive columns over banks.
    static constexpr int pad(int p) {
        // lane-tail units read the last pass column-fast (lane = q + 16 r):
        // two elements per row keep those reads on distinct banks
        if (LANE && p + 2 == NP) return 2;
        return (p + 1 < NP && log_m(p + 1) < 5) ? (1 << log_m(p + 1)) : 0;
    }
    static constexpr int padded(int p) {
        return (1 << LOG_NU) + ((1 << LOG_NU) >> log_m(p)) * pad(p);
    }
    static constexpr int region() {
        int r = 1 << LOG_NU;
        for (int p = 0; p + 1 < NP; ++p) r = padded(p) > r ? padded(p) : r;
        return r | 1;   // odd stride between units
    }
    // LDS of an exchange done in two rounds (half of the rows each)
    static constexpr int half_region() {
        int r = 0;
        for (int p = 0; p + 1 < NP; ++p) r = padded(p) / 2 > r ? padded(p) / 2 : r;
        return r;
    }
};

// Exchanges in two rounds: a whole-transform unit (one per workgroup) writes
// and reads half of the exchange's rows per round where its exchange would not
// fit in LDS (binary16 2^16 points: 256 KiB of data, 128-135 KiB per round),
// and also where halving the exchange lets more workgroups share a CU whose
// one-round occupancy is below the 16 waves that lanes holding 256 bytes or
// more of data leave registers for (binary16 2^15 points on 512 lanes: one
// workgroup of 135 KiB or two of 70 KiB; binary32 2^14 on 256 lanes; binary32
// 2^13 on 256 lanes: two workgroups or four).  Each pass after an exchange
// must hold at least two groups per lane (the rounds split a lane's groups in
// halves).
constexpr size_t kLdsBytes = 160 * 1024;
template <class E, int LOG_E, int MODE, int UPW, class PP>
constexpr int exchange_rounds() {
    if (!(MODE == MODE_SMALL && UPW == 1 && PP::NP > 1))
        return 1;
    for (int p = 1; p < PP::NP; ++p)
        if (PP::lr(p) >= LOG_E) return 1;
    const size_t one = (size_t)PP::region() * sizeof(E), two = (size_t)PP::half_region() * sizeof(E);
    if (one > kLdsBytes) return 2;
    if ((sizeof(E) << LOG_E) < 256) return 1;
    const int lanes = 1 << (PP::log_nu - LOG_E);
    const int waves = lanes >= 64 ? lanes / 64 : 1;
    const int wg1 = (int)(kLdsBytes / one), wg2 = (int)(kLdsBytes / two);
    return (wg1 * waves < 16 && wg2 > wg1) ? 2 : 1;
}
// LDS elements of a workgroup.
template <class E, int LOG_E, int MODE, int UPW, class PP>
constexpr size_t unit_lds_elems() {
    return exchange_rounds<E, LOG_E, MODE, UPW, PP>() == 2 ? (size_t)PP::half_region()
                                                           : (size_t)UPW * PP::region();
}
// Twiddles held in LDS (configurations with PIPE = 3).  In a unit whose table
// offsets are its own (whole transforms and column units: q0 = 0, no level
// shift), pass P >= 1 (span L0 before it, radix R) takes for group column
// q < L0 the entries q + L0 c of the level-ordered table, 1 <= c < R: the
// contiguous entries [L0, L0 R), and passes 1 .. P together take [L0_1,
// L0_P R_P).  The workgroup copies that run into LDS once, after the exchange
// area, and the passes read it there instead of through the vector memory
// path, where many lanes would fetch the same entries: the middle pass of a
// three-pass whole transform (all lanes of a column), and every pass after
// the first of a column unit (its lanes run the same groups of UPW columns).
// A whole transform's last pass reads distinct entries per lane (NU/2 of
// them) and keeps its table loads under PIPE = 3; PIPE = 4 copies those too
// (every pass after the first reads LDS: the run [L0_1, NU), for transforms
// small enough that it fits beside the exchange).  Under PIPE = 3 a middle
// pass whose column is the same across a wave loads through the scalar cache
// (group_twiddles) instead.
template <int LOG_NU, int LOG_E, int MODE, int LANE, class PP, int PIPE>
constexpr int lds_twiddle_last_pass() {
    if (LANE || (PIPE != 3 && PIPE != 4 && PIPE != 5)) return 0;
    if (MODE == MODE_COLS || (MODE == MODE_SMALL && PIPE == 4)) return PP::NP >= 2 ? PP::NP - 1 : 0;
    if (MODE != MODE_SMALL || PP::NP != 3) return 0;
    constexpr int G = (1 << LOG_NU) >> LOG_E;
    if (PP::log_m(1) >= 6 && G % 64 == 0) return 0;
    return 1;
}
template <int LOG_NU, int LOG_E, int MODE, int LANE, class PP, int PIPE>
constexpr int lds_twiddle_entries() {
    constexpr int LAST = lds_twiddle_last_pass<LOG_NU, LOG_E, MODE, LANE, PP, PIPE>();
    if (LAST == 0) return 0;
    return (1 << (PP::log_l0(LAST) + PP::lr(LAST))) - (1 << PP::log_l0(1));
}
// Row units (PIPE = 3): the first pass of row q0 takes entries
// q0 + c 2^log_m, 1 <= c < R0, the same for the G lanes of the unit; the
// workgroup copies entry (c, unit) to LDS slot (c - 1) UPW + unit.
template <int MODE, int UPW, class PP, int PIPE>
constexpr int lds_row_twiddle_entries() {
    return (MODE == MODE_ROWS && PIPE == 3) ? ((1 << PP::lr(0)) - 1) * UPW : 0;
}
// Byte offset of the twiddle copy: the exchange area rounded up to 16 bytes.
template <class E, int LOG_E, int MODE, int UPW, class PP>
constexpr size_t lds_twiddle_offset() {
    return (unit_lds_elems<E, LOG_E, MODE, UPW, PP>() * sizeof(E) + 15) / 16 * 16;
}
// LDS bytes of a workgroup: the exchange area, and with PIPE = 3, 4 or 5 the twiddle copy.
template <class E, int LOG_NU, int LOG_E, int MODE, int UPW, int LANE, int PIPE, class PP, int ENC = ENC_TABLE>
constexpr size_t unit_lds_bytes() {
    constexpr int TE = lds_twiddle_entries<LOG_NU, LOG_E, MODE, LANE, PP, PIPE>() +
                       lds_row_twiddle_entries<MODE, UPW, PP, PIPE>();
    if (TE == 0) return unit_lds_elems<E, LOG_E, MODE, UPW, PP>() * sizeof(E);
    return lds_twiddle_offset<E, LOG_E, MODE, UPW, PP>() + (size_t)TE * sizeof(TwT<E, ENC>);
}
// Whether a configuration fits a workgroup's LDS for element type E (the
// configuration list serves both element sizes; entries that do not fit are
// neither compiled nor offered).  PIPE = 3, 4 and 5 also need a pass to serve.
template <class E, int LOG_NU, int LOG_E, int MODE, int UPW, int LANE, int PIPE, class PP, int ENC = ENC_TABLE>
constexpr bool unit_fits() {
    if ((PIPE == 3 || PIPE == 4 || PIPE == 5) && lds_twiddle_entries<LOG_NU, LOG_E, MODE, LANE, PP, PIPE>() == 0 &&
        lds_row_twiddle_entries<MODE, UPW, PP, PIPE>() == 0)
        return false;
    return unit_lds_bytes<E, LOG_NU, LOG_E, MODE, UPW, LANE, PIPE, PP, ENC>() <= kLdsBytes;
}

// ------------------------------------------------------------------ the kernel

// Geometry of one unit inside its transform.
struct UnitGeom {
    int64_t base_in, base_out, in_stride, out_stride;
    int q0, log_lb;
};

template <int LOG_NU, int MODE>
__device__ __forceinline__ UnitGeom unit_geom(int64_t unit, int log_m) {
    UnitGeom u;
    u.in_stride = u.out_stride = 1;
    u.q0 = 0;
    u.log_lb = 0;
    if (MODE == MODE_SMALL) {
        u.base_in = u.base_out = unit << LOG_NU;
    } else if (MODE == MODE_COLS) {
        const int64_t b = unit >> log_m;
        const int64_t r0 = unit & ((int64_t(1) << log_m) - 1);
        u.base_in = u.base_out = (b << (log_m + LOG_NU)) + r0;
        u.in_stride = u.out_stride = int64_t(1) << log_m;
    } else {
        const int64_t b = unit >> log_m;
        u.q0 = (int)(unit & ((int64_t(1) << log_m) - 1));
        u.log_lb = log_m;
        u.base_in = (b << (log_m + LOG_NU)) + ((int64_t)u.q0 << LOG_NU);
        u.base_out = (b << (log_m + LOG_NU)) + u.q0;
        u.out_stride = int64_t(1) << log_m;
    }
    return u;
}

// 16-byte vector used for staged global <-> LDS copies.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Copies elements [first, first + count) of `in` into lds[0, count) with
// 16-byte non-temporal loads (count and first are multiples of 16 bytes;
// the global pointer is 16-byte aligned), then waits for the whole block.
template <class E, int NT, int CAP>
__device__ __forceinline__ void stage_in(const E* in, E* lds, int64_t first, int64_t count) {
    constexpr int VEC = 16 / (int)sizeof(E);
    static_assert(CAP % (VEC * NT) == 0, "block must split into 16-byte vectors per thread");
    const u32x4_t* src = reinterpret_cast<const u32x4_t*>(in + first);
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(lds);
    const int nvec = (int)(count / VEC);
#pragma unroll
    for (int k = 0; k < CAP / VEC / NT; ++k) {
        const int j = k * NT + (int)threadIdx.x;
        if (j < nvec) dst[j] = __builtin_nontemporal_load(src + j);
    }
    __syncthreads();
}

// Copies lds[0, count) to elements [first, first + count) of `out` with
// 16-byte non-temporal stores.
template <class E, int NT, int CAP>
__device__ __forceinline__ void stage_out(const E* lds, E* out, int64_t first, int64_t count) {
    constexpr int VEC = 16 / (int)sizeof(E);
    static_assert(CAP % (VEC * NT) == 0, "block must split into 16-byte vectors per thread");
    const u32x4_t* src = reinterpret_cast<const u32x4_t*>(lds);
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(out + first);
    const int nvec = (int)(count / VEC);
#pragma unroll
    for (int k = 0; k < CAP / VEC / NT; ++k) {
        const int j = k * NT + (int)threadIdx.x;
        if (j < nvec) __builtin_nontemporal_store(src[j], dst + j);
    }
}

// ------------------------------------------------------- cross-lane stages

// Exchanges the upper half (D = 32) or the odd rows (D = 16) of x with the
// lower half / even rows of y (v_permlane32_swap / v_permlane16_swap).
// Afterwards every lane l holds, in (x, y), the pair (x_lower, x_upper) of
// lanes (l & ~D, l | D) when l is a lower lane, and (y_lower, y_upper) when
// l is an upper lane: both operands of one butterfly whose partners are D
// lanes apart.
template <int D>
__device__ __forceinline__ void swap_halves(uint32_t& x, uint32_t& y) {
    if constexpr (D == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    } else {
        static_assert(D == 16, "lane distance 16 or 32");
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    }
}
template <int D>
__device__ __forceinline__ void swap_halves(f2_t& x, f2_t& y) {
    uint32_t x0 = __builtin_bit_cast(uint32_t, (float)x.x), x1 = __builtin_bit_cast(uint32_t, (float)x.y);
    uint32_t y0 = __builtin_bit_cast(uint32_t, (float)y.x), y1 = __builtin_bit_cast(uint32_t, (float)y.y);
    swap_halves<D>(x0, y0);
    swap_halves<D>(x1, y1);
    x.x = __builtin_bit_cast(float, x0);
    x.y = __builtin_bit_cast(float, x1);
    y.x = __builtin_bit_cast(float, y0);
    y.y = __builtin_bit_cast(float, y1);
}

// The last two radix-2 stages of a one-wave unit of NU points, across lanes.
// On entry lane (u, r, q) = (bit 5, bit 4, bits 0-3) holds v[e] = Y[r'][q + 16 e]
// with r' = 2u + r (the four residues left) for e < NU/64.
//   Stage with span NU/2 pairs residues r' and r' + 2 (lanes 32 apart): after
//   swapping register pairs (v[2k], v[2k+1]), lane (u, r, q) holds a = Y[r][j],
//   b = Y[r + 2][j] with j = q + 16 (2k + u); A -> v[2k] (= Y'[r][j]),
//   B -> v[2k+1] (= Y'[r][j + NU/4]).
//   Stage with span NU pairs residues 0 and 1 (lanes 16 apart): the lane with
//   r = 0 takes the pair of register v[2k], the lane with r = 1 that of v[2k+1];
//   the column is jb = q + 16 (2k + u) + (NU/4) r; A -> X[jb], B -> X[jb + NU/2].
// Every butterfly keeps its operands, table entry (level-ordered index
// L/2 + j) and FMA order, so the result equals the radix-2 Stockham definition.
template <class E, int LOG_NU>
__device__ __forceinline__ void lane_tail(E* v, const typename TwOf<E>::type* __restrict__ lt,
                                          int lane) {
    using TW = typename TwOf<E>::type;
    constexpr int NU = 1 << LOG_NU;
    constexpr int EL = NU / 64;
    const int q = lane & 15, r = (lane >> 4) & 1, u = lane >> 5;
    TW tw[EL / 2];
#pragma unroll
    for (int k = 0; k < EL / 2; ++k) tw[k] = lt[NU / 4 + q + 16 * (2 * k + u)];
#pragma unroll
    for (int k = 0; k < EL / 2; ++k) {
        swap_halves<32>(v[2 * k], v[2 * k + 1]);
        bfly(v[2 * k], v[2 * k + 1], tw[k]);
    }
#pragma unroll
    for (int k = 0; k < EL / 2; ++k) tw[k] = lt[NU / 2 + q + 16 * (2 * k + u) + (NU / 4) * r];
#pragma unroll
    for (int k = 0; k < EL / 2; ++k) {
        swap_halves<16>(v[2 * k], v[2 * k + 1]);
        bfly(v[2 * k], v[2 * k + 1], tw[k]);
    }
}

// Where the units of one workgroup live: a regular launch takes UPW
// consecutive units per workgroup (GridGeo); the uneven-batch kernel takes the
// units of one work item (BatchGeo, in fft_batch.hpp).
template <bool TWPF, int ENC = ENC_TABLE, int TWL = 0>
struct GridGeoT {
    // the next pass's twiddles are loaded a pass ahead (twiddle_prefetch)
    static constexpr bool kTwiddlePrefetch = TWPF;
    // passes read their twiddles from an LDS copy: 0 none, else the PIPE
    // value that decides which (lds_twiddle_last_pass)
    static constexpr int kTwiddleLds = TWL;
    // leading table entries held in LDS just below the exchange area (none)
    static constexpr int kTwiddlePrefix = 0;
    // the butterfly's path encoding (bfly_enc)
    static constexpr int kEncoding = ENC;
    // a workgroup's units are consecutive in memory (block_first, block_units)
    static constexpr bool kBlockRsrc = true;
    int64_t ublk, units;
    int log_m;
    int lane_id;       // threadIdx.x (opaque per block in the persistent loop)
    template <int LOG_NU, int MODE>
    __device__ __forceinline__ UnitGeom get(int ul) const {
        return unit_geom<LOG_NU, MODE>(ublk + ul, log_m);
    }
    __device__ __forceinline__ bool active(int ul) const { return ublk + ul < units; }
    __device__ __forceinline__ int tid() const { return lane_id; }
    // staging: the workgroup's units are elements [first, first + count)
    __device__ __forceinline__ int64_t block_first(int log_nu) const { return ublk << log_nu; }
    __device__ __forceinline__ int64_t block_units(int upw) const {
        return units - ublk < upw ? units - ublk : upw;
    }
};
using GridGeo = GridGeoT<false>;

// Lanes and units.  A lane holds groups of UPL units (units per lane): the
// same group positions g + G u of units ul0 .. ul0 + UPL - 1, so each twiddle
// it loads serves all of them.  Its registers hold unit k's elements at
// v[k * EL .. k * EL + EL).  Column units and the row kernel's last pass map
// consecutive lanes to consecutive units ("unit-fast", UPL = 1 only); every
// other pass maps consecutive lanes to consecutive groups of one unit.

// Pass-0 inputs of this lane straight from HBM (unstaged configurations):
// group r = g + G u (residue r, span 1) takes elements r + M i, i < R.
// The streaming hint is used only where a wave's accesses cover whole lines:
// per instruction the G lanes of a unit read G consecutive elements, so where
// those fill a 128-byte line (elsewhere the line's other elements come with
// the lane's later loads and must still be cached then).
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int LANE,
          class Geo, class SI>
__device__ __forceinline__ void load_pass0(E* v, const SI* in, const Geo& gp) {
    using PP = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
    constexpr int NU = 1 << LOG_NU;
    constexpr int EL = 1 << LOG_E;
    constexpr int G = NU / EL;
    constexpr int R = 1 << PP::lr(0);
    constexpr int M = 1 << PP::log_m(0);
    constexpr int GPL = EL / R;
    constexpr bool unit_fast = (MODE == MODE_COLS);
    const int tid = gp.tid();
    const int ul0 = unit_fast ? (tid % UPW) : (tid / G) * UPL;
    const int g = unit_fast ? (tid / UPW) : (tid % G);
    if constexpr (MODE == MODE_SMALL && Geo::kBlockRsrc && NU * sizeof(SI) > 4096) {
        const rsrc_t rs = block_rsrc(in + gp.block_first(LOG_NU), gp.block_units(UPW) << LOG_NU);
#pragma unroll
        for (int k = 0; k < UPL; ++k) {
            E* vk = v + k * EL;
            if (gp.active(ul0 + k)) {
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const uint32_t lane_off = (uint32_t)(((ul0 + k) * NU + g + G * u) * (int)sizeof(SI));
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        vk[u * R + i] = buf_load<true, E, SI>(rs, lane_off, (uint32_t)(M * i * (int)sizeof(SI)));
                }
            } else {
#pragma unroll
                for (int e = 0; e < EL; ++e) vk[e] = E{};
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < UPL; ++k) {
        E* vk = v + k * EL;
        if (gp.active(ul0 + k)) {
            const UnitGeom geo = gp.template get<LOG_NU, MODE>(ul0 + k);
#pragma unroll
            for (int u = 0; u < GPL; ++u) {
                const int r = g + G * u;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int64_t idx = r + (int64_t)M * i;
                    vk[u * R + i] = load_elem<MODE != MODE_COLS && G * (int)sizeof(SI) >= 128, E>(in + geo.base_in + idx * geo.in_stride);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < EL; ++e) vk[e] = E{};
        }
    }
}

// Twiddles of register pass P for this lane's groups: tw[u * R + c] is the
// entry of butterfly index c (1 <= c < R) of group g + G u.  Entries depend on
// the lane's position only, not on data.
// (group_twiddles: the same for one group, tw[c].)
template <class E, int LOG_NU, int LOG_E, int MODE, int LR0, int LR1, int LR2, int LANE, int P,
          int ENC = ENC_TABLE>
__device__ __forceinline__ void group_twiddles(TwT<E, ENC>* tw, const TwT<E, ENC>* __restrict__ lt,
                                               const UnitGeom& geo0, int g, int u) {
    using PP = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
    constexpr int NU = 1 << LOG_NU;
    constexpr int EL = 1 << LOG_E;
    constexpr int G = NU / EL;
    constexpr int R = 1 << PP::lr(P);
    constexpr int L0 = 1 << PP::log_l0(P);
    constexpr int LOGM = PP::log_m(P);
    const int q = (g + G * u) >> LOGM;        // column within the unit
    // Radix-4 form: its stages read entries c = S + e < 2S <= R/2 only, and
    // entry 0 is the span-2 stage's radix-2 butterfly.
    constexpr int C0 = ENC == ENC_RADIX4 ? 0 : 1;
    constexpr int C1 = ENC == ENC_RADIX4 ? R / 2 : R;
    if constexpr (P == 0 && MODE != MODE_ROWS) {
#pragma unroll
        for (int c = C0; c < C1; ++c) tw[c] = lt[c];
    } else if constexpr (MODE == MODE_SMALL && !LANE && LOGM >= 6 && G % 64 == 0) {
        // A wave's 64 lanes hold 64 consecutive groups (g = tid mod G, G a
        // multiple of 64), and with M >= 64 groups per column they share the
        // column q: the entries are wave-uniform and load through the scalar
        // cache, which keeps them off the vector memory path.
        const int qs = __builtin_amdgcn_readfirstlane(q);
#pragma unroll
        for (int c = C0 > 0 ? C0 : 1; c < C1; ++c) tw[c] = lt[qs + L0 * c];
    } else {
        const int qg = geo0.q0 + (q << geo0.log_lb);
        const int lg0 = L0 << geo0.log_lb;
#pragma unroll
        for (int c = C0 > 0 ? C0 : 1; c < C1; ++c) tw[c] = lt[qg + lg0 * c];
    }
}
template <class E, int LOG_NU, int LOG_E, int MODE, int LR0, int LR1, int LR2, int LANE, int P,
          int ENC = ENC_TABLE>
__device__ __forceinline__ void pass_twiddles(TwT<E, ENC>* tw, const TwT<E, ENC>* __restrict__ lt,
                                              const UnitGeom& geo0, int g) {
    using PP = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
    constexpr int R = 1 << PP::lr(P);
    constexpr int GPL = (1 << LOG_E) / R;
#pragma unroll
    for (int u = 0; u < GPL; ++u)
        group_twiddles<E, LOG_NU, LOG_E, MODE, LR0, LR1, LR2, LANE, P, ENC>(tw + u * R, lt, geo0, g, u);
}

// Twiddle prefetch (configurations with PIPE = 2): whole-transform units load
// the twiddles of pass P + 1 at the start of pass P, so that their latency
// overlaps the data loads (pass 0) or the exchange; the table misses the
// vector L1 cache, and loaded at the point of use each pass waits for L2.  It
// costs the VGPRs that hold them, so it is a per-configuration choice for the
// tuner; it applies where each pass's set fits in 64 VGPRs per lane.
template <class E, int LOG_NU, int LOG_E, int MODE, int LR0, int LR1, int LR2, int LANE>
constexpr bool twiddle_prefetch() {
    using PP = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
    if (MODE != MODE_SMALL || LANE || PP::NP < 2) return false;
    for (int p = 1; p < PP::NP; ++p) {
        const int regs = ((1 << LOG_E) >> PP::lr(p)) * ((1 << PP::lr(p)) - 1) *
                         (int)(sizeof(typename TwOf<E>::type) / 4);
        if (regs > 64) return false;
    }
    return true;
}

// Copies table entries [0, T) into LDS at dst (16-byte aligned), 16 bytes per
// lane per step, for NT lanes; the caller's next barrier publishes them.
template <class TW, int T, int NT>
__device__ __forceinline__ void copy_table_prefix(const TW* __restrict__ lt, unsigned char* dst) {
    constexpr int CHUNKS = (int)(T * sizeof(TW) / 16);
    static_assert((T * sizeof(TW)) % 16 == 0, "whole 16-byte chunks");
    const uint4* src = reinterpret_cast<const uint4*>(lt);
    uint4* d = reinterpret_cast<uint4*>(dst);
#pragma unroll
    for (int i = (int)threadIdx.x; i < CHUNKS; i += NT) d[i] = src[i];
}

// Marks a prefetched twiddle as needed here: the loads that fill it must have
// returned by this point (and the compiler cannot move them after it).
__device__ __forceinline__ void pin_twiddle(TwH& t) { asm volatile("" : "+v"(t.w), "+v"(t.ts)); }
__device__ __forceinline__ void pin_twiddle(TwF& t) {
    asm volatile("" : "+v"(t.sm), "+v"(t.m), "+v"(t.t), "+v"(t.mask));
}

// One register pass P of the unit schedule: gather (global or LDS), twiddles,
// LR radix-2 stages per group, scatter (LDS or global).  twp: this pass's
// twiddles when the previous pass loaded them (twiddle_prefetch).
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PRE, int P, class Geo, class SI, class SO>
__device__ __forceinline__ void unit_pass(E* v, E* lds, const TwT<E, Geo::kEncoding>* __restrict__ lt,
                                          const SI* in, SO* out, const Geo& gp,
                                          const TwT<E, Geo::kEncoding>* twp = nullptr) {
    using TW = TwT<E, Geo::kEncoding>;
    using PP = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
    constexpr int NP = PP::NP;
    if constexpr (P < NP) {
        constexpr int NU = 1 << LOG_NU;
        constexpr int EL = 1 << LOG_E;
        constexpr int G = NU / EL;
        constexpr int RS = PP::region();
        constexpr int LR = PP::lr(P);
        constexpr int R = 1 << LR;
        constexpr int L0 = 1 << PP::log_l0(P);
        constexpr int LOGM = PP::log_m(P);
        constexpr int M = 1 << LOGM;
        constexpr int GPL = EL / R;
        constexpr int NT_OF = (UPW / UPL) * G;
        constexpr bool unit_fast = (MODE == MODE_COLS) || (MODE == MODE_ROWS && P == NP - 1);
        static_assert(UPL == 1 || (MODE == MODE_SMALL && !LANE && UPW % UPL == 0),
                      "several units per lane: whole-transform units without the lane tail");
        static_assert(!STG || !LANE || (sizeof(SI) == sizeof(E) && sizeof(SO) == sizeof(E)),
                      "the lane tail's staging copies stored values unchanged");
        constexpr int XR = exchange_rounds<E, LOG_E, MODE, UPW, PP>();
        static_assert(XR == 1 || (UPL == 1 && !LANE && !STG && PRE == 0),
                      "two-round exchanges: one plain unit per workgroup");
        const int tid = gp.tid();
        const int ul0 = unit_fast ? (tid % UPW) : (tid / G) * UPL;
        const int g0 = unit_fast ? (tid / UPW) : (tid % G);
        // lane-tail units: the last pass takes group (r, q) on lane q + 16 r
        constexpr bool lane_map = LANE && P == NP - 1;
        const int g = lane_map ? (((g0 & 15) << 2) | (g0 >> 4)) : g0;
        // twiddle offsets of the row kernel (the same for every unit of a lane)
        const UnitGeom geo0 = gp.template get<LOG_NU, MODE>(ul0);

        // ---- the next pass's twiddles (whole-transform units), issued ahead of
        // this pass's gather; the empty asm keeps them ahead of it
        // (passes served from an LDS copy of the table neither prefetch nor
        // take prefetched twiddles)
        constexpr bool PF = Geo::kTwiddlePrefetch && !PRE &&
                            twiddle_prefetch<E, LOG_NU, LOG_E, MODE, LR0, LR1, LR2, LANE>();
        constexpr int TWL_LAST = lds_twiddle_last_pass<LOG_NU, LOG_E, MODE, LANE, PP, Geo::kTwiddleLds>();
        constexpr bool TWL = P >= 1 && P <= TWL_LAST;
        constexpr bool PFN = PF && P + 1 < NP && !(P + 1 <= TWL_LAST);   // prefetch pass P + 1's
        constexpr bool PFU = PF && P > 0 && !TWL;                         // use this pass's prefetch
        // table entries [0, TPX) held in LDS just below the exchange area
        // (persistent and list kernels): a pass P >= 1 of a unit with its own
        // table offsets whose entries q + L0 c all lie below TPX reads them there
        constexpr int TPX = Geo::kTwiddlePrefix;
        constexpr bool TWX = !TWL && !PFU && TPX > 0 && P >= 1 && MODE != MODE_ROWS && (L0 << LR) <= TPX;
        constexpr int NEXT_TW = PFN ? (EL >> PP::lr(P + 1)) << PP::lr(P + 1) : 1;
        TW twn[NEXT_TW];
        if constexpr (PFN) {
            pass_twiddles<E, LOG_NU, LOG_E, MODE, LR0, LR1, LR2, LANE, P + 1, Geo::kEncoding>(twn, lt, geo0, g);
            asm volatile("" ::: "memory");
        }

        // binary16-storage plans (binary32 butterflies): pass 0 keeps the stored
        // pairs for its first stage (bfly_stored), which widens them inside
        // its FMAs
        constexpr bool STORED0 = P == 0 && !PRE && !STG && std::is_same_v<E, f2_t> &&
                                 std::is_same_v<SI, uint32_t> && Geo::kEncoding == ENC_TABLE;
        uint32_t raw[STORED0 ? (UPL << LOG_E) : 1];

        // ---- gather
        if constexpr (P == 0 && STG) {
            // The workgroup's units are contiguous in memory (whole transforms,
            // or consecutive rows of the workspace): copy the block into LDS
            // (natural order) with 16-byte streaming loads, then gather the
            // pass's decimated groups from LDS.
            // (stored values: widened as they are gathered where storage and
            // compute precision differ)
            SI* lds_in = reinterpret_cast<SI*>(lds);
            stage_in<SI, NT_OF, UPW << LOG_NU>(in, lds_in, gp.block_first(LOG_NU),
                                               gp.block_units(UPW) << LOG_NU);
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                const SI* nat = lds_in + (ul0 + k) * NU;
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const int r = g + G * u;
#pragma unroll
                    for (int i = 0; i < R; ++i) v[k * EL + u * R + i] = to_compute(nat[r + M * i], E{});
                }
            }
        } else if constexpr (STORED0) {
            load_pass0<uint32_t, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, LANE>(raw, in, gp);
        } else if constexpr (P == 0) {
            if constexpr (!PRE) load_pass0<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, LANE>(v, in, gp);
        } else if constexpr (XR == 2) {
            // gathered by the previous pass's two-round exchange
        } else {
            constexpr int PADP = PP::pad(P - 1);
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                const E* reg = lds + (ul0 + k) * RS;
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const int gam = g + G * u;
                    const int r = gam & (M - 1);
                    const int q = gam >> LOGM;
                    // local index r + M i + (NU/L0) q lives in row q of the exchange
                    const int basep = r + ((NU / L0) + PADP) * q;
#pragma unroll
                    for (int i = 0; i < R; ++i) v[k * EL + u * R + i] = reg[basep + M * i];
                }
            }
        }

        // ---- twiddles (once per group position) and stages (for each unit)
#pragma unroll
        for (int u = 0; u < GPL; ++u) {
            TW tw[R];
            if constexpr (PFU) {
#pragma unroll
                for (int c = 1; c < R; ++c) tw[c] = twp[u * R + c];
            } else if constexpr (TWL) {
                // entry q + L0 c of the table sits at q + L0 c - L0_1 of the copy
                constexpr int L01 = 1 << PP::log_l0(1);
                const TW* ltw = reinterpret_cast<const TW*>(reinterpret_cast<const unsigned char*>(lds) +
                                                            lds_twiddle_offset<E, LOG_E, MODE, UPW, PP>());
                const int q = (g + G * u) >> LOGM;
#pragma unroll
                for (int c = 1; c < R; ++c) tw[c] = ltw[q + L0 * c - L01];
            } else if constexpr (P == 0 && MODE == MODE_ROWS && Geo::kTwiddleLds == 3) {
                const TW* ltw = reinterpret_cast<const TW*>(reinterpret_cast<const unsigned char*>(lds) +
                                                            lds_twiddle_offset<E, LOG_E, MODE, UPW, PP>());
#pragma unroll
                for (int c = 1; c < R; ++c) tw[c] = ltw[(c - 1) * UPW + ul0];
            } else if constexpr (TWX) {
                const TW* ltp = reinterpret_cast<const TW*>(reinterpret_cast<const unsigned char*>(lds) -
                                                            (size_t)TPX * sizeof(TW));
                const int q = (g + G * u) >> LOGM;
#pragma unroll
                for (int c = 1; c < R; ++c) tw[c] = ltp[q + L0 * c];
            } else {
                group_twiddles<E, LOG_NU, LOG_E, MODE, LR0, LR1, LR2, LANE, P, Geo::kEncoding>(tw, lt, geo0, g, u);
            }
            // radix-4 form: the first pass of an odd log2 N starts with the span-2 stage
            constexpr bool ODD = Geo::kEncoding == ENC_RADIX4 && P == 0 && (LOG_NU & 1);
            if constexpr (STORED0) {
                // stage 1 of the pass pairs element i with i + R/2 under entry 1
#pragma unroll
                for (int k = 0; k < UPL; ++k) {
                    E* vg = v + k * EL + u * R;
                    const uint32_t* rg = raw + k * EL + u * R;
#pragma unroll
                    for (int i = 0; i < R / 2; ++i) bfly_stored(rg[i], rg[i + R / 2], tw[1], vg[i], vg[i + R / 2]);
                    reg_pass<LR, Geo::kEncoding, ODD, 2>(vg, tw);
                }
            } else {
#pragma unroll
                for (int k = 0; k < UPL; ++k) reg_pass<LR, Geo::kEncoding, ODD>(v + k * EL + u * R, tw);
            }
        }
        if constexpr (PFN) {
            // entries c >= 1 of each group are the loaded ones
#pragma unroll
            for (int i = 0; i < NEXT_TW; ++i)
                if (i & ((1 << PP::lr(P + 1)) - 1)) pin_twiddle(twn[i]);
        }

        // ---- scatter
        if constexpr (LANE && P == NP - 1) {
            static_assert(G == 64 && GPL == 1 && M == 4 && L0 == 16 && MODE == MODE_SMALL,
                          "lane tail needs one wave per unit and a 16 x 4 last pass");
            lane_tail<E, LOG_NU>(v, lt, g0);
            // lane (u, r, q) holds X[jb] in v[2k] and X[jb + NU/2] in v[2k+1],
            // jb = q + 16 (2k + u) + (NU/4) r
            const int q = g0 & 15, r = (g0 >> 4) & 1, u = g0 >> 5;
            if constexpr (STG) {
                __syncthreads();
                E* nat = lds + ul0 * NU;
#pragma unroll
                for (int k = 0; k < EL / 2; ++k) {
                    const int jb = q + 16 * (2 * k + u) + (NU / 4) * r;
                    nat[jb] = v[2 * k];
                    nat[jb + NU / 2] = v[2 * k + 1];
                }
                __syncthreads();
                stage_out<E, NT_OF, UPW << LOG_NU>(lds, out, gp.block_first(LOG_NU),
                                                   gp.block_units(UPW) << LOG_NU);
            } else if (gp.active(ul0)) {
#pragma unroll
                for (int k = 0; k < EL / 2; ++k) {
                    const int jb = q + 16 * (2 * k + u) + (NU / 4) * r;
                    store_elem<true>(v[2 * k], out + geo0.base_out + jb);
                    store_elem<true>(v[2 * k + 1], out + geo0.base_out + jb + NU / 2);
                }
            }
        } else if constexpr (P + 1 < NP && XR == 2) {
            // Two rounds over the exchange's NR = L0 R rows: round h moves rows
            // [h NR/2, (h+1) NR/2).  The rows a lane writes in round h are its
            // elements e in [h R/2, (h+1) R/2) (row q + L0 e, q < L0); the rows
            // the next pass reads in round h are those of its groups
            // u1 in [h GPL1/2, (h+1) GPL1/2) (row q1 = (g + G u1) / M1 <
            // NR/2 exactly when u1 < GPL1/2).  So each lane moves half of its
            // registers per round, and the next pass's values go to a second
            // array until every value of this pass has been written.
            constexpr int PAD = PP::pad(P);
            constexpr int NR = L0 * R;
            constexpr int R1 = 1 << PP::lr(P + 1);
            constexpr int LOGM1 = PP::log_m(P + 1);
            constexpr int M1 = 1 << LOGM1;
            constexpr int GPL1 = EL / R1;
            static_assert(GPL1 >= 2 && R >= 2 && UPW == 1, "two-round exchange: halves of groups and rows");
            E w[EL];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h > 0 || P > 0) __syncthreads();   // readers of LDS are done
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const int gam = g + G * u;
                    const int r = gam & (M - 1);
                    const int q = gam >> LOGM;
#pragma unroll
                    for (int e = h * (R / 2); e < (h + 1) * (R / 2); ++e)
                        lds[r + (M + PAD) * (q + L0 * e - h * (NR / 2))] = v[u * R + e];
                }
                __syncthreads();
#pragma unroll
                for (int u1 = h * (GPL1 / 2); u1 < (h + 1) * (GPL1 / 2); ++u1) {
                    const int gam1 = g + G * u1;
                    const int r1 = gam1 & (M1 - 1);
                    const int q1 = gam1 >> LOGM1;
                    const int basep = r1 + (M + PAD) * (q1 - h * (NR / 2));
#pragma unroll
                    for (int i = 0; i < R1; ++i) w[u1 * R1 + i] = lds[basep + M1 * i];
                }
            }
#pragma unroll
            for (int i = 0; i < EL; ++i) v[i] = w[i];
        } else if constexpr (P + 1 < NP) {
            constexpr int PAD = PP::pad(P);
            if constexpr (P > 0 || STG) __syncthreads();   // readers of LDS are done
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                E* reg = lds + (ul0 + k) * RS;
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const int gam = g + G * u;
                    const int r = gam & (M - 1);
                    const int q = gam >> LOGM;
                    // local index r + M (q + L0 e) lives in row q + L0 e
#pragma unroll
                    for (int e = 0; e < R; ++e)
                        reg[r + (M + PAD) * (q + L0 * e)] = v[k * EL + u * R + e];
                }
            }
            __syncthreads();
        } else if constexpr (STG && MODE == MODE_SMALL) {
            // outputs to LDS in natural order, then 16-byte streaming stores
            // (row units stage only their input: their outputs are strided)
            // (rounded to the storage precision as they are written)
            __syncthreads();                      // every lane is done reading LDS
            SO* lds_out = reinterpret_cast<SO*>(lds);
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                SO* nat = lds_out + (ul0 + k) * NU;
#pragma unroll
                for (int u = 0; u < GPL; ++u) {
                    const int q = g + G * u;
#pragma unroll
                    for (int e = 0; e < R; ++e) nat[q + L0 * e] = to_storage(v[k * EL + u * R + e], SO{});
                }
            }
            __syncthreads();
            stage_out<SO, NT_OF, UPW << LOG_NU>(lds_out, out, gp.block_first(LOG_NU),
                                                gp.block_units(UPW) << LOG_NU);
        } else if constexpr (MODE == MODE_SMALL && Geo::kBlockRsrc && NU * sizeof(SO) > 4096) {
            const rsrc_t rs = block_rsrc(out + gp.block_first(LOG_NU), gp.block_units(UPW) << LOG_NU);
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                if (gp.active(ul0 + k)) {
#pragma unroll
                    for (int u = 0; u < GPL; ++u) {
                        const int q = g + G * u;  // M = 1: every group is a column
                        const uint32_t lane_off = (uint32_t)(((ul0 + k) * NU + q) * (int)sizeof(SO));
#pragma unroll
                        for (int e = 0; e < R; ++e)
                            buf_store<true, E, SO>(v[k * EL + u * R + e], rs, lane_off,
                                                   (uint32_t)(L0 * e * (int)sizeof(SO)));
                    }
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < UPL; ++k) {
                if (gp.active(ul0 + k)) {
                    const UnitGeom geo = gp.template get<LOG_NU, MODE>(ul0 + k);
#pragma unroll
                    for (int u = 0; u < GPL; ++u) {
                        const int q = g + G * u;  // M = 1: every group is a column
#pragma unroll
                        for (int e = 0; e < R; ++e) {
                            const int64_t idx = q + (int64_t)L0 * e;
                            // streaming only where one instruction's elements fill whole lines:
                            // G consecutive ones of a whole transform (as load_pass0), or the
                            // row kernel's UPW consecutive rows
                            store_elem<(MODE == MODE_SMALL && G * (int)sizeof(SO) >= 128) ||
                                       (MODE == MODE_ROWS && UPW * (int)sizeof(SO) >= 128)>(v[k * EL + u * R + e],
                                                           out + geo.base_out + idx * geo.out_stride);
                        }
                    }
                }
            }
        }
        unit_pass<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PRE, P + 1>(v, lds, lt, in,
                                                                                           out, gp, twn);
    }
}

// in/out: element pointers (uint32_t = binary16 pair, f2_t = binary32 pair).
// lt: level-ordered table.  units: units in this launch.  log_m: log2(N/NU),
// the number of columns (MODE_COLS) or rows (MODE_ROWS) per transform; 0 for
// MODE_SMALL.  Dynamic LDS: UPW * PassPlan::region() elements.
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE, class SI, class SO, int ENC>
__device__ __forceinline__ void unit_kernel_body(const SI* in, SO* out, const TwT<E, ENC>* __restrict__ lt,
                                                 int64_t units, int log_m);

// SI, SO: storage types of the input and output (E unless the plan stores
// binary16 and computes in binary32).
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE, class SI = E, class SO = E, int ENC = ENC_TABLE>
__global__ void __launch_bounds__((UPW / UPL) << (LOG_NU - LOG_E))
fft_unit_kernel(const SI* in, SO* out, const TwT<E, ENC>* __restrict__ lt, int64_t units, int log_m) {
    unit_kernel_body<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE, SI, SO, ENC>(
        in, out, lt, units, log_m);
}

// The pipelined kernel holds two register sets; the compiler is asked to fit
// three waves per SIMD so the prefetch is not bought with occupancy.
template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE, class SI = E, class SO = E, int ENC = ENC_TABLE>
__global__ void __launch_bounds__((UPW / UPL) << (LOG_NU - LOG_E)) __attribute__((amdgpu_waves_per_eu(3)))
fft_unit_kernel_pipe(const SI* in, SO* out, const TwT<E, ENC>* __restrict__ lt, int64_t units, int log_m) {
    unit_kernel_body<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, PIPE, SI, SO, ENC>(
        in, out, lt, units, log_m);
}

template <class E, int LOG_NU, int LOG_E, int UPW, int UPL, int MODE, int LR0, int LR1, int LR2, int STG,
          int LANE, int PIPE, class SI, class SO, int ENC>
__device__ __forceinline__ void unit_kernel_body(const SI* in, SO* out, const TwT<E, ENC>* __restrict__ lt,
                                                 int64_t units, int log_m) {
    static_assert(LR0 + LR1 + LR2 + 2 * LANE == LOG_NU, "radices must multiply to NU");
    static_assert(LR0 <= LOG_E && LR1 <= LOG_E && LR2 <= LOG_E, "radix above elements per lane");
    static_assert(MODE != MODE_ROWS || LR1 > 0, "row units need two passes");
    static_assert(STG == 0 || MODE != MODE_COLS, "staging needs contiguous units");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    E* lds = reinterpret_cast<E*>(lds_raw);
    static_assert(PIPE != 1 || (STG == 0 && MODE == MODE_SMALL), "pipelining needs unstaged units");
    static_assert((PIPE != 2 && PIPE != 5) || MODE == MODE_SMALL, "twiddle prefetch needs whole-transform units");
    static_assert((PIPE != 4 && PIPE != 5) || MODE != MODE_ROWS,
                  "LDS twiddles of later passes need units with their own table offsets");
    static_assert(ENC != ENC_RADIX4 ||
                      (MODE == MODE_SMALL && !LANE && PIPE != 1 && PIPE != 2 && PIPE != 5 &&
                       LR0 % 2 == LOG_NU % 2 && LR1 % 2 == 0 && LR2 % 2 == 0),
                  "radix-4 form: whole transforms whose passes start on radix-4 stage boundaries");
    E v[UPL << LOG_E];
    if constexpr (PIPE == 1) {
        // persistent: this workgroup takes blocks blockIdx.x, + gridDim.x, ...
        // in two register sets used alternately (a and b), so the next block's
        // HBM reads are in flight while the current block is computed and no
        // register copy forces an early wait
        E vb[UPL << LOG_E];
        const int64_t nblk = (units + UPW - 1) / UPW;
        const int64_t step = gridDim.x;
        int64_t blk = blockIdx.x;
        // The thread index is re-read through an empty asm statement for each
        // block, so index arithmetic is recomputed per block instead of being
        // hoisted out of the loop and held in registers throughout it.
        auto geo = [&](int64_t b) {
            int t = (int)threadIdx.x;
            asm volatile("" : "+v"(t));
            return GridGeo{b * UPW, units, log_m, t};
        };
        if (blk < nblk)
            load_pass0<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, LANE>(
                v, in, geo(blk));
        while (blk < nblk) {
            if (blk + step < nblk)
                load_pass0<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, LANE>(
                    vb, in, geo(blk + step));
            unit_pass<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, 1, 0>(
                v, lds, lt, in, out, geo(blk));
            __syncthreads();    // LDS is reused by the next block
            blk += step;
            if (blk >= nblk) break;
            if (blk + step < nblk)
                load_pass0<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, LANE>(
                    v, in, geo(blk + step));
            unit_pass<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, 1, 0>(
                vb, lds, lt, in, out, geo(blk));
            __syncthreads();
            blk += step;
        }
    } else {
        if constexpr (PIPE == 3 && MODE == MODE_ROWS) {
            // row units: entry (c, unit) of the first pass, one 8- or 16-byte
            // entry per lane per step; the first pass reads them right after
            // its loads, so a barrier publishes them
            using PPT = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
            using TW = TwT<E, ENC>;
            constexpr int TE = lds_row_twiddle_entries<MODE, UPW, PPT, PIPE>();
            constexpr int NT = (UPW / UPL) << (LOG_NU - LOG_E);
            TW* dst = reinterpret_cast<TW*>(lds_raw + lds_twiddle_offset<E, LOG_E, MODE, UPW, PPT>());
            const int64_t ublk = (int64_t)blockIdx.x * UPW;
            for (int i = (int)threadIdx.x; i < TE; i += NT) {
                const int c = 1 + i / UPW, ul = i % UPW;
                const UnitGeom geo = unit_geom<LOG_NU, MODE>(ublk + ul, log_m);   // q0 < 2^log_m
                dst[i] = lt[geo.q0 + ((int64_t)c << geo.log_lb)];
            }
            __syncthreads();
        } else if constexpr (PIPE == 3 || PIPE == 4 || PIPE == 5) {
            // copy the table run of the passes served from LDS (from L0 of
            // pass 1 on) after the exchange area, 16 bytes per lane per step;
            // the barrier after the first exchange's writes orders it before
            // pass 1 reads it
            using PPT = PassPlan<LOG_NU, LR0, LR1, LR2, LANE>;
            using TW = TwT<E, ENC>;
            constexpr int TE = lds_twiddle_entries<LOG_NU, LOG_E, MODE, LANE, PPT, PIPE>();
            constexpr int CHUNKS = (int)(TE * sizeof(TW) / 16);
            constexpr int NT = (UPW / UPL) << (LOG_NU - LOG_E);
            static_assert(TE > 0 && (TE * sizeof(TW)) % 16 == 0 && ((1 << LR0) * sizeof(TW)) % 16 == 0,
                          "LDS twiddles: whole 16-byte chunks from a 16-byte aligned start");
            const uint4* src = reinterpret_cast<const uint4*>(lt + (1 << LR0));
            uint4* dst = reinterpret_cast<uint4*>(lds_raw + lds_twiddle_offset<E, LOG_E, MODE, UPW, PPT>());
            for (int i = (int)threadIdx.x; i < CHUNKS; i += NT) dst[i] = src[i];
        }
        // PIPE = 5: the middle pass from LDS (as PIPE = 3) and the last pass's
        // twiddles prefetched a pass ahead (as PIPE = 2)
        constexpr int TWL = (PIPE == 3 || PIPE == 4 || PIPE == 5) ? PIPE : 0;
        const GridGeoT<PIPE == 2 || PIPE == 5, ENC, TWL> gp{(int64_t)blockIdx.x * UPW, units, log_m,
                                                             (int)threadIdx.x};
        unit_pass<E, LOG_NU, LOG_E, UPW, UPL, MODE, LR0, LR1, LR2, STG, LANE, 0, 0>(v, lds, lt, in, out,
                                                                               gp);
    }
}

}  // namespace dsfft
