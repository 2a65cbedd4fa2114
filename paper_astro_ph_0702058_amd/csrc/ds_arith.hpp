// ds_arith.hpp -- double-single (float-float) arithmetic for gfx950.
//
// A value is the unevaluated sum hi + lo of two floats with |lo| <= ulp(hi)/2, about 48
// significant bits.  Built from error-free transformations:
//   two_sum       Knuth (TAOCP vol. 2): s = fl(a + b) and the exact rounding error e.
//   fast_two_sum  Dekker (1971): the same when |a| >= |b|, three operations.
//   two_prod      p = fl(a * b) and e = fma(a, b, -p), exact with a fused multiply-add.
// The additions follow the two variants of Hida, Li & Bailey's double-double library: the
// "accurate" form renormalises after adding the low parts with their own error term; the
// "sloppy" form adds the low parts plainly.  The reciprocal square root starts from the
// hardware single-precision estimate and applies one correction step of third order,
// y = y0 (1 + r/2 + 3 r^2/8) with r = 1 - s y0^2 evaluated in double-single.
//
// The library is compiled with -ffp-contract=off so that no a*b+c in this file is fused
// behind the algorithms' backs; every fused multiply-add here is written explicitly.
#pragma once

#include <hip/hip_runtime.h>

namespace nbody {

struct ds {
    float hi, lo;
};

__device__ __forceinline__ ds ds_make(float h, float l) { return ds{h, l}; }
__device__ __forceinline__ ds ds_from_float(float a) { return ds{a, 0.0f}; }

__device__ __forceinline__ ds two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return ds{s, e};
}

__device__ __forceinline__ ds fast_two_sum(float a, float b) {
    const float s = a + b;
    const float e = b - (s - a);
    return ds{s, e};
}

__device__ __forceinline__ ds two_prod(float a, float b) {
    const float p = a * b;
    const float e = __builtin_fmaf(a, b, -p);
    return ds{p, e};
}

// Accurate addition: error below about 2^-47 of the result, also under cancellation.
__device__ __forceinline__ ds ds_add(ds a, ds b) {
    ds s = two_sum(a.hi, b.hi);
    const ds t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ds ds_neg(ds a) { return ds{-a.hi, -a.lo}; }
__device__ __forceinline__ ds ds_sub(ds a, ds b) { return ds_add(a, ds_neg(b)); }

// Sloppy addition: cheaper; relative error bounded by the operands' magnitudes rather than the
// result's, adequate where no catastrophic cancellation is expected.
__device__ __forceinline__ ds ds_add_sloppy(ds a, ds b) {
    ds s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ds ds_mul(ds a, ds b) {
    ds p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fmaf(a.hi, b.lo, p.lo);
    p.lo = __builtin_fmaf(a.lo, b.hi, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

// The same products before their final renormalisation: hi + lo is exactly the sum that
// ds_mul / ds_sqr / ds_mul_f return (fast_two_sum is error-free), with |lo| up to about two
// units in the last place of hi.  Such a value may feed an addition, which renormalises its
// own result, or another product, whose neglected lo * lo term stays below about 2^-44 of it.
__device__ __forceinline__ ds ds_mul_raw(ds a, ds b) {
    ds p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fmaf(a.hi, b.lo, p.lo);
    p.lo = __builtin_fmaf(a.lo, b.hi, p.lo);
    return p;
}

__device__ __forceinline__ ds ds_sqr_raw(ds a) {
    ds p = two_prod(a.hi, a.hi);
    p.lo = __builtin_fmaf(a.hi + a.hi, a.lo, p.lo);
    return p;
}

__device__ __forceinline__ ds ds_mul_f_raw(ds a, float b) {
    ds p = two_prod(a.hi, b);
    p.lo = __builtin_fmaf(a.lo, b, p.lo);
    return p;
}

__device__ __forceinline__ ds ds_mul_f(ds a, float b) {
    ds p = two_prod(a.hi, b);
    p.lo = __builtin_fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ds ds_sqr(ds a) {
    ds p = two_prod(a.hi, a.hi);
    p.lo = __builtin_fmaf(a.hi + a.hi, a.lo, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

// s^(-1/2) for s > 0.
__device__ __forceinline__ ds ds_rsqrt(ds s) {
    const float y0 = __builtin_amdgcn_rsqf(s.hi);
    const ds y0sq = two_prod(y0, y0);
    const ds t = ds_mul(s, y0sq);                 // ~ 1
    const float r = (1.0f - t.hi) - t.lo;        // 1 - t.hi is exact (Sterbenz)
    const float corr = y0 * (r * __builtin_fmaf(0.375f, r, 0.5f));
    return fast_two_sum(y0, corr);
}

__device__ __forceinline__ double ds_to_double(ds a) { return (double)a.hi + (double)a.lo; }

__device__ __forceinline__ ds ds_from_double(double d) {
    const float h = (float)d;
    return ds{h, (float)(d - (double)h)};
}

}  // namespace nbody
