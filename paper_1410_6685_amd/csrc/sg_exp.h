// Correctly rounded binary32 exp for the fused element-wise kernels (host and device).
//
// The chain semantics round every float32 node to nearest-even (an element function's
// result is the binary32 nearest to the exact value), so exp must be correctly rounded:
// a filter threshold downstream of exp (x > 0.1 after exp(-u^2)) turns any 1-ulp error into
// a different element count.
//
// Method (table-driven reduction after Tang, ACM TOMS 15(2), 1989, evaluated in float64):
//   k = rint(t * 32/ln2), r = t - k*ln2/32 (|r| <= ln2/64), j = k mod 32, m = floor(k/32),
//   exp(t) = 2^m * 2^(j/32) * exp(r),  exp(r) - 1 by its degree-6 Taylor polynomial.
// The float64 result y has relative error below 2^-50.  If y lies farther than 2^-46*y
// from every binary32 rounding boundary, RN32(y) = RN32(exp t).  Otherwise (about one
// element in 2^22) the value is recomputed in double-double arithmetic (about 2^-100
// relative error) with the Taylor series to degree 13, which settles the rounding since
// exp of a nonzero binary32 is never a rounding boundary.
#pragma once
#include <cmath>
#include <cstdint>

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

// Fast path: returns RN32(exp t) and hard = false, or hard = true when t needs the
// double-double path.
SG_HD float exp_rn_fast(float t, bool& hard) {
    hard = false;
    if (t != t) return t;
    if (t >= u2f(SG_EXP_OVF_BITS)) return __builtin_inff();
    if (t <= u2f(SG_EXP_UNF_BITS)) return 0.0f;
    const double td = (double)t;
    const double kd = rint(td * SG_EXP_INV_L);
    const int k = (int)kd;
    const int j = k & 31;
    const int m = k >> 5;
    double r = fma(-kd, SG_EXP_L1, td);
    r = fma(-kd, SG_EXP_L2, r);
    double q = fma(r, SG_EXP_IFACT_HI[6], SG_EXP_IFACT_HI[5]);
    q = fma(q, r, SG_EXP_IFACT_HI[4]);
    q = fma(q, r, SG_EXP_IFACT_HI[3]);
    q = fma(q, r, SG_EXP_IFACT_HI[2]);
    q = fma(q, r, 1.0);
    const double p = q * r;  // exp(r) - 1
    const double T = SG_EXP_TAB_HI[j];
    const double y = fma(T, p, T) * pow2d(m);
    const float f = (float)y;
    const double diff = y - (double)f;
    const double dist = fabs(fabs(diff) - half_gap(f2u(f), diff));
    hard = dist <= y * 0x1p-46;
    return f;
}

// Correctly rounded binary32 exp.  *slow (if given) is incremented when the double-double
// path was taken.
SG_HD float exp_rn(float t, int* slow = nullptr) {
    bool hard;
    const float f = exp_rn_fast(t, hard);
    if (!hard) return f;
    if (slow) ++*slow;
    return exp_rn_slow(t);
}

}  // namespace sgx
