// Attenuation factors of one voxel segment, for the GPU kernels (and a
// host build used only to test them).
//
// For the optical thickness x = Sigma * l >= 0 of a segment the score of
// Eq. 1 needs em = 1 - exp(-x) (accurate also for tiny x) and the weight
// leaving the voxel needs g = exp(-x) (accurate also for large x).  Forming
// one from the other loses everything where it matters (1 + expm1(-x) for
// x >> 1, 1 - exp(-x) for x << 1), and two library calls cost two
// exponentials.  Both come here from a single evaluation:
//
//   1. Cody and Waite's argument reduction: -x = k ln2 + r, |r| <= ln2/2,
//      with ln2 split into a head whose product with k is exact and a tail;
//   2. q = expm1(r) from its Taylor series in Horner form (degree 13 for
//      double, 7 for float: the truncation is below a quarter ulp for
//      |r| <= 0.347);
//   3. g = 2^k (1 + q) and em = (1 - 2^k) - 2^k q, each one fused
//      multiply-add (both results are then within a few ulp).
//
// The split constants are ln2 rounded to 53 (24) bits with the low 21 (12)
// bits cleared, and the rest of ln2 rounded to the working precision.
#pragma once

#ifndef VRC_HD
#if defined(__HIPCC__)
#define VRC_HD __host__ __device__
#else
#define VRC_HD
#endif
#endif

#include <cmath>

namespace vrc {

template <typename R>
struct AttenConst;

template <>
struct AttenConst<double> {
    static constexpr double inv_ln2 = 1.4426950408889634;
    static constexpr double ln2_hi = 0.6931471804855391;
    static constexpr double ln2_lo = 7.440617110012397e-11;
    static constexpr double x_max = 708.0;  // exp(-x) below the normal range beyond this
    static constexpr int degree = 13;
};

template <>
struct AttenConst<float> {
    static constexpr float inv_ln2 = 1.44269502f;
    static constexpr float ln2_hi = 0.693115234375f;
    static constexpr float ln2_lo = 3.194618329871446e-05f;
    static constexpr float x_max = 87.0f;
    static constexpr int degree = 7;
};

// 1/j!, exact factorial in double (j <= 18), rounded once.
VRC_HD constexpr double inv_factorial(int j)
{
    double f = 1.0;
    for (int i = 2; i <= j; ++i) f *= static_cast<double>(i);
    return 1.0 / f;
}

VRC_HD inline double vrc_fma(double a, double b, double c) { return ::fma(a, b, c); }
VRC_HD inline float vrc_fma(float a, float b, float c) { return ::fmaf(a, b, c); }
VRC_HD inline double vrc_ldexp(double a, int k) { return ::ldexp(a, k); }
VRC_HD inline float vrc_ldexp(float a, int k) { return ::ldexpf(a, k); }
VRC_HD inline double vrc_rint(double a) { return ::rint(a); }
VRC_HD inline float vrc_rint(float a) { return ::rintf(a); }

// The Horner sum p = 1/1! + r (1/2! + ... + r / D!) of the expm1 series.
// In FP64 device code (D = 13) it is one block of twelve dependent
// three-operand FMAs: left to itself the compiler keeps the coefficients in
// vector registers and uses the two-operand FMA, which overwrites its
// addend, so every step first copies a coefficient (twelve copies per
// evaluation).  The arithmetic is the same sequence of fused multiply-adds.
template <typename R>
VRC_HD inline R horner_series(R r)
{
    R p = static_cast<R>(inv_factorial(AttenConst<R>::degree));
#pragma unroll
    for (int j = AttenConst<R>::degree - 1; j >= 1; --j) p = vrc_fma(p, r, static_cast<R>(inv_factorial(j)));
    return p;
}
VRC_HD inline float horner_expm1(float r) { return horner_series(r); }
static_assert(AttenConst<double>::degree == 13, "the FP64 Horner block below has twelve steps");
VRC_HD inline double horner_expm1(double r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double p;
    asm("v_fma_f64 %0, %2, %1, %3\n\t"
        "v_fma_f64 %0, %0, %1, %4\n\t"
        "v_fma_f64 %0, %0, %1, %5\n\t"
        "v_fma_f64 %0, %0, %1, %6\n\t"
        "v_fma_f64 %0, %0, %1, %7\n\t"
        "v_fma_f64 %0, %0, %1, %8\n\t"
        "v_fma_f64 %0, %0, %1, %9\n\t"
        "v_fma_f64 %0, %0, %1, %10\n\t"
        "v_fma_f64 %0, %0, %1, %11\n\t"
        "v_fma_f64 %0, %0, %1, %12\n\t"
        "v_fma_f64 %0, %0, %1, %13\n\t"
        "v_fma_f64 %0, %0, %1, %14"
        : "=&v"(p)
        : "v"(r), "v"(inv_factorial(13)), "v"(inv_factorial(12)), "v"(inv_factorial(11)), "v"(inv_factorial(10)),
          "v"(inv_factorial(9)), "v"(inv_factorial(8)), "v"(inv_factorial(7)), "v"(inv_factorial(6)),
          "v"(inv_factorial(5)), "v"(inv_factorial(4)), "v"(inv_factorial(3)), "v"(inv_factorial(2)),
          "v"(inv_factorial(1)));
    return p;
#else
    return horner_series(r);
#endif
}

// g = exp(-x), em = 1 - exp(-x) for x >= 0 (x > x_max or NaN: g = 0, em = 1).
// Branch-free: out-of-range arguments are evaluated at 0 and their results
// replaced, so the lanes of a wavefront never split here.
template <typename R>
VRC_HD inline void attenuation(R x, R &g, R &em)
{
    using C = AttenConst<R>;
    const bool big = !(x <= C::x_max);
    const R y = big ? R(0) : -x;
    const R kf = vrc_rint(y * C::inv_ln2);
    R r = vrc_fma(-kf, C::ln2_hi, y);
    r = vrc_fma(-kf, C::ln2_lo, r);
    // Horner: q = r (1/1! + r (1/2! + r (1/3! + ... + r / degree!)))
    const R q = horner_expm1(r) * r;
    const R s = vrc_ldexp(R(1), static_cast<int>(kf));
    const R gv = vrc_fma(s, q, s);
    const R ev = vrc_fma(-s, q, R(1) - s);
    g = big ? R(0) : gv;
    em = big ? R(1) : ev;
}

}  // namespace vrc
