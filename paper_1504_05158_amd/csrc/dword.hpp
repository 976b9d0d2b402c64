// Error-free transformations and double-word ("float-float") arithmetic in
// binary32, so that the velocity update needs no binary64 on the device.
//
//  two_sum       Knuth's TwoSum: s = fl(a + b), e = a + b - s exactly (any a, b).
//  fast_two_sum  Dekker's Fast2Sum: the same when |a| >= |b| (or a = 0).
//  two_prod      p = fl(a b), e = a b - p exactly, from one fused multiply-add
//                (exact as long as a b does not underflow).
//  dw_add_f      double-word + float, Algorithm 4 (DWPlusFP) of Joldes,
//                Muller & Popescu, "Tight and rigorous error bounds for basic
//                building blocks of double-word arithmetic", ACM TOMS 44(2),
//                2017: relative error at most 2u^2 (u = 2^-24).
//  dw_add        double-word + double-word, their Algorithm 6
//                (AccurateDWPlusDW): relative error at most 3u^2 / (1 - 4u),
//                relative to the exact sum, so it stays accurate when the
//                operands cancel.
//
// Every operation below is written out with explicit roundings; the library
// is compiled without floating-point contraction, so the compiler fuses
// nothing behind these sequences' backs.
#pragma once
#include <hip/hip_runtime.h>

namespace qap {

struct DW {
    float hi, lo;  // value hi + lo, |lo| <= ulp(hi) / 2
};

__device__ __forceinline__ DW two_sum(float a, float b)
{
    const float s = __fadd_rn(a, b);
    const float bb = __fsub_rn(s, a);
    const float aa = __fsub_rn(s, bb);
    const float e = __fadd_rn(__fsub_rn(a, aa), __fsub_rn(b, bb));
    return DW{s, e};
}

__device__ __forceinline__ DW fast_two_sum(float a, float b)
{
    const float s = __fadd_rn(a, b);
    const float e = __fsub_rn(b, __fsub_rn(s, a));
    return DW{s, e};
}

__device__ __forceinline__ DW two_prod(float a, float b)
{
    const float p = __fmul_rn(a, b);
    return DW{p, __builtin_fmaf(a, b, -p)};
}

__device__ __forceinline__ DW dw_add_f(DW x, float y)
{
    const DW s = two_sum(x.hi, y);
    const float v = __fadd_rn(x.lo, s.lo);
    return fast_two_sum(s.hi, v);
}

__device__ __forceinline__ DW dw_add(DW x, DW y)
{
    const DW s = two_sum(x.hi, y.hi);
    const DW t = two_sum(x.lo, y.lo);
    const float c = __fadd_rn(s.lo, t.hi);
    const DW v = fast_two_sum(s.hi, c);
    const float w = __fadd_rn(t.lo, v.lo);
    return fast_two_sum(v.hi, w);
}

__device__ __forceinline__ DW dw_neg(DW x) { return DW{-x.hi, -x.lo}; }

}  // namespace qap
