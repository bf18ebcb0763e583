// sin x and cos x of one float64 argument, for the kernels' per-coordinate
// tables (Ackley's cos(2 pi x) and its derivative, Fletcher-Powell's sin x and
// cos x).
//
// Method: Cody-Waite reduction x = k pi/2 + r, k = nearest integer to
// x 2/pi, with pi/2 split into P1 = pi/2 rounded to float64 and
// P2 = (pi/2 - P1) rounded; each product k P sits inside an FMA, so r carries
// one rounding per step (the split's own remainder, about 1.5e-33 per unit of
// k, is far below that).  On |r| <= pi/4 the Taylor series of sin through
// r^17 and of cos through r^16 (the first omitted terms are below 1e-19
// there), evaluated by Horner's rule in r^2; the quadrant k mod 4 swaps and
// negates the pair.  Arguments beyond kFastTrigMax take the library's sincos,
// whose reduction stays exact for any finite x.
#pragma once

#include <hip/hip_runtime.h>

namespace chessfad {

constexpr double kFastTrigMax = 65536.0;
constexpr double kTwoOverPi = 0.63661977236758134308;   // 2 / pi
constexpr double kHalfPi1 = 1.5707963267948966;         // pi/2 rounded to float64
constexpr double kHalfPi2 = 6.123233995736766e-17;      // pi/2 - kHalfPi1, rounded

// 1 / k!, exact factorials (17! < 2^53)
constexpr double inv_fact(int k) {
    double f = 1.0;
    for (int j = 2; j <= k; ++j) f *= j;
    return 1.0 / f;
}

// the library's routine, out of line: its reduction for large arguments
// needs registers that the fast path does not
inline __host__ __device__ __attribute__((noinline)) double2 cf_sincos_large(double x) {
    double s, c;
    sincos(x, &s, &c);
    return make_double2(s, c);
}

__host__ __device__ __forceinline__ void cf_sincos(double x, double* s, double* c) {
    if (!(fabs(x) <= kFastTrigMax)) {
        const double2 sc = cf_sincos_large(x);
        *s = sc.x;
        *c = sc.y;
        return;
    }
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kHalfPi1, x);
    r = fma(-k, kHalfPi2, r);
    const double z = r * r;
    // sin r = r + r z (-1/3! + z (1/5! - ...)), cos r = 1 + z (-1/2! + z (1/4! - ...))
    double ps = inv_fact(17);
    ps = fma(ps, z, -inv_fact(15));
    ps = fma(ps, z, inv_fact(13));
    ps = fma(ps, z, -inv_fact(11));
    ps = fma(ps, z, inv_fact(9));
    ps = fma(ps, z, -inv_fact(7));
    ps = fma(ps, z, inv_fact(5));
    ps = fma(ps, z, -inv_fact(3));
    double pc = inv_fact(16);
    pc = fma(pc, z, -inv_fact(14));
    pc = fma(pc, z, inv_fact(12));
    pc = fma(pc, z, -inv_fact(10));
    pc = fma(pc, z, inv_fact(8));
    pc = fma(pc, z, -inv_fact(6));
    pc = fma(pc, z, inv_fact(4));
    pc = fma(pc, z, -0.5);
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z, pc, 1.0);
    const int q = (int)k;
    const double s1 = (q & 1) ? cr : sr;
    const double c1 = (q & 1) ? -sr : cr;
    *s = (q & 2) ? -s1 : s1;
    *c = (q & 2) ? -c1 : c1;
}

}  // namespace chessfad
