// Correctly rounded binary32 exp for the fused element-wise kernels (host and device).
//
// The chain semantics round every float32 node to nearest-even (an element function's
// result is the binary32 nearest to the exact value), so exp must be correctly rounded:
// a filter threshold downstream of exp (x > 0.1 after exp(-u^2)) turns any 1-ulp error into
// a different element count.
//
// Method (table-driven reduction after Tang, ACM TOMS 15(2), 1989, evaluated in float64):
//   k = rint(t * 256/ln2), r = t - k*ln2/256 (|r| <= ln2/512), j = k mod 256,
//   m = floor(k/256), exp(t) = 2^m * 2^(j/256) * exp(r),  exp(r) - 1 by its degree-3
//   Taylor polynomial (a larger table buys two fewer polynomial steps per element).
// The float64 result y has relative error below 1.44e-13.  If y lies clearly away from every
// binary32 rounding boundary (checked on its low mantissa bits), RN32(y) = RN32(exp t).
// Otherwise (about one element in 2^17) the value is recomputed in double-double arithmetic
// (about 2^-100 relative error; 32 intervals, Taylor series to degree 13), which settles
// the rounding since exp of a nonzero binary32 is never a rounding boundary.
#pragma once
#ifndef __HIPCC_RTC__
#include <cmath>
#endif
#ifndef __HIPCC_RTC__
#include <cstdint>
#else
// run-time compilation: fixed-width types without the C library headers
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
typedef unsigned long uintptr_t;
#endif

#include "sg_exp_table.h"

#ifndef SG_HD
#define SG_HD __host__ __device__ __forceinline__
#endif

namespace sgx {

SG_HD uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
SG_HD float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }
SG_HD double u2d(uint64_t u) { return __builtin_bit_cast(double, u); }

// 2^e as a double for -1022 <= e <= 1023
SG_HD double pow2d(int e) { return u2d((uint64_t)(e + 1023) << 52); }

struct dd { double hi, lo; };

SG_HD dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
SG_HD dd fast_two_sum(double a, double b) {  // requires |a| >= |b|
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
SG_HD dd two_prod(double a, double b) {
    double p = a * b;
    return {p, fma(a, b, -p)};
}
SG_HD dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
SG_HD dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}

// Half the binary32 spacing on the side of `diff` around the binary32 value with bits fb.
SG_HD double half_gap(uint32_t fb, double diff) {
    uint32_t E = (fb >> 23) & 0xFFu;
    double ulp = (E == 0) ? pow2d(-149) : pow2d((int)E - 150);
    if (diff < 0.0 && (fb & 0x7FFFFFu) == 0 && E > 1) ulp *= 0.5;
    return 0.5 * ulp;
}

// Round the double-double value H + L (positive, within binary32 range) to binary32.
SG_HD float round_dd_to_f32(double H, double L) {
    float f = (float)H;
    double diff = (H - (double)f) + L;  // H - f is exact
    uint32_t fb = f2u(f);
    double h = half_gap(fb, diff);
    double ad = fabs(diff);
    if (ad > h || (ad == h && (fb & 1u)))
        fb = diff > 0.0 ? fb + 1u : fb - 1u;
    return u2f(fb);
}

// Rarely taken (about once in 2^20 elements); callers run it after the fast path so that
// it is not unrolled with it.
SG_HD float exp_rn_slow(float t) {
    const double td = (double)t;
    const double kd = rint(td * SG_EXP_INV_L);
    const int k = (int)kd;
    const int j = k & 31;
    const int m = k >> 5;
    double r1 = fma(-kd, SG_EXP_L1, td);  // exact: k*L1 has at most 53 bits
    dd p2 = two_prod(kd, SG_EXP_L2);
    dd r = two_sum(r1, -p2.hi);
    r.lo = (r.lo - p2.lo) - kd * SG_EXP_L3;
    r = fast_two_sum(r.hi, r.lo);
    dd q = {SG_EXP_IFACT_HI[13], SG_EXP_IFACT_LO[13]};
    for (int i = 12; i >= 1; --i)
        q = dd_add(dd_mul(q, r), dd{SG_EXP_IFACT_HI[i], SG_EXP_IFACT_LO[i]});
    dd e = dd_mul(q, r);  // exp(r) - 1
    dd T = {SG_EXP_TAB_HI[j], SG_EXP_TAB_LO[j]};
    dd res = dd_add(T, dd_mul(T, e));
    double s = pow2d(m);
    return round_dd_to_f32(res.hi * s, res.lo * s);
}

// The 29 bits of y below binary32 precision lie within 2048 units of the half-way pattern
// 2^28: low29 in [2^28 - 2048, 2^28 + 2048].  Shifted left by 3 (the three bits above them
// drop out) and offset, that is one unsigned comparison:
// (low29 * 8 - (2^31 - 16384)) mod 2^32 <= 32768.
SG_HD bool near_half(double y) {
    const uint32_t lo = (uint32_t)__builtin_bit_cast(uint64_t, y);
    return (lo << 3) + (16384u - 0x80000000u) <= 32768u;
}

// Fast path: returns RN32(exp t) and hard = false, or hard = true when t needs the
// double-double path.  `tab` is SG_EXPF_TAB (2^(j/256)); kernels pass a copy in LDS.
//
// k is rounded to an integer by adding 1.5*2^52 (its low 32 bits are then k in two's
// complement), r = t - k*ln2/256 is exact up to the F2 term (|r| <= ln2/512 + 2^-40 <
// 1.36e-3), and exp(r) - 1 is its degree-3 Taylor polynomial, whose truncation is below
// r^4/24 * 1.001 < 1.44e-13.  With the float64 roundings of r, the polynomial, the table
// entry and the product (each 2^-53 relative), the result y is within 1.44e-13 relative of
// exp(t), i.e. within 2^10.4 < 1300 units of its last place (y < 2^(e+1) for y in
// [2^e, 2^(e+1))), so RN32(y) = RN32(exp t) unless the 29 bits below binary32 precision
// lie within 2048 units of the half-way pattern 2^28 (about one argument in 2^17).
// Results below the binary32 normal range take the slow path (their rounding position
// differs).
// The float64 core alone, for an ordinary argument: -87 <= t < the overflow threshold.
SG_HD float exp_rn_core(float t, const double* tab, bool& hard);

// The core in two stages, so that a caller can issue the table reads of several elements before
// it evaluates their polynomials: the reduction gives the table index (k mod 256) and the
// rounded multiple; the finish combines the table entry with exp(r) - 1.
struct ExpCore {
    double td, sh;
    int idx;
};
SG_HD ExpCore exp_core_reduce(float t) {
    ExpCore c;
    c.td = (double)t;
    c.sh = fma(c.td, SG_EXPF_INV_L, 0x1.8p52);
    c.idx = (int)(uint32_t)__builtin_bit_cast(uint64_t, c.sh) & ((1 << SG_EXPF_BITS) - 1);
    return c;
}
SG_HD float exp_core_finish(const ExpCore& c, double T, bool& hard) {
    const int k = (int)(uint32_t)__builtin_bit_cast(uint64_t, c.sh);
    const double kd = c.sh - 0x1.8p52;
    double r = fma(-kd, SG_EXPF_L1, c.td);
    r = fma(-kd, SG_EXPF_L2, r);
    const double q = fma(r, 1.0 / 6.0, 0.5);
    const double p = fma(q, r * r, r);  // exp(r) - 1
    const double y = __builtin_ldexp(fma(T, p, T), k >> SG_EXPF_BITS);  // exact: the result is a normal double
    hard = near_half(y);
    return (float)y;
}
SG_HD float exp_rn_core(float t, const double* tab, bool& hard) {
    const ExpCore c = exp_core_reduce(t);
    return exp_core_finish(c, tab[c.idx], hard);
}

// an argument the core handles (NaN fails both comparisons)
SG_HD bool exp_ordinary(float t) { return t >= -87.0f && t < u2f(SG_EXP_OVF_BITS); }

SG_HD float exp_rn_fast(float t, const double* tab, bool& hard) {
    // Branch-free: the core runs on t clamped into [-87, 89] (where k fits and 2^(k>>6) is a
    // normal double), then the special cases select their own result.
    const float tc = __builtin_fminf(__builtin_fmaxf(t, -87.0f), 89.0f);
    const double td = (double)tc;
    const double sh = fma(td, SG_EXPF_INV_L, 0x1.8p52);
    const int k = (int)(uint32_t)__builtin_bit_cast(uint64_t, sh);
    const double kd = sh - 0x1.8p52;
    double r = fma(-kd, SG_EXPF_L1, td);
    r = fma(-kd, SG_EXPF_L2, r);
    const double q = fma(r, 1.0 / 6.0, 0.5);
    const double p = fma(q, r * r, r);  // exp(r) - 1
    const double T = tab[k & ((1 << SG_EXPF_BITS) - 1)];
    const double y = fma(T, p, T) * pow2d(k >> SG_EXPF_BITS);
    // exp(t) < 2^-125.5 (t < -87) is near or below the binary32 normal range: slow path
    const bool special = t != t || t >= u2f(SG_EXP_OVF_BITS) || t <= u2f(SG_EXP_UNF_BITS);
    hard = !special && (t < -87.0f || near_half(y));
    float f = (float)y;
    f = t <= u2f(SG_EXP_UNF_BITS) || t < -87.0f ? 0.0f : f;
    f = t >= u2f(SG_EXP_OVF_BITS) ? __builtin_inff() : f;
    f = t != t ? t : f;
    return f;
}

// Correctly rounded binary32 exp.  *slow (if given) is incremented when the double-double
// path was taken.
SG_HD float exp_rn(float t, int* slow = nullptr) {
    bool hard;
    const float f = exp_rn_fast(t, SG_EXPF_TAB, hard);
    if (!hard) return f;
    if (slow) ++*slow;
    return exp_rn_slow(t);
}

}  // namespace sgx
