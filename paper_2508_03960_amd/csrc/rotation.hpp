// Rotation coefficients of one raster step (Eq. A2), shared by the plain
// stepper and the per-isochromat transition composition.
#pragma once

#include <hip/hip_runtime.h>

namespace gbs {

// Rotation coefficients of one step:
//   a = sin(theta)/|B| = -gdt * S(q),  b = (1 - cos theta)/|B|^2 = gdt^2 * C(q),
//   S(q) = sum_n (-q)^n / (2n+1)!,  C(q) = sum_n (-q)^n / (2n+2)!,  q = theta^2.
// For q <= 1/16 six terms of each series reach double precision, for q <= 1
// ten (n <= 9); larger angles use sqrt and sincos.  FP64 throughout.
// One Horner step r = q S + c as a single VOP3 FMA with the coefficient c in
// a scalar register pair.  Left to itself the compiler picks the two-address
// v_fmac_f64, whose addend is its destination, and then copies the constant
// into that register at every step: two instructions per term.
__device__ __forceinline__ double horner(double q, double S, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(q), "v"(S), "s"(c));
    return r;
}

// First Horner step q a + b with both coefficients in scalar registers: a
// multiply and an add, which keeps no vector register busy with a constant
// (one FMA would need one of them in a vector register pair for the whole
// kernel, at the price of occupancy).
__device__ __forceinline__ double horner_first(double q, double a, double b) {
    double r;
    asm("v_mul_f64 %0, %1, %2\n\tv_add_f64 %0, %0, %3" : "=&v"(r) : "v"(q), "s"(a), "s"(b));
    return r;
}

struct Series {
    static __device__ __forceinline__ void coeffs(double q, double &S, double &C) {
        S = horner_first(q, 8.2206352466243297e-18, -2.8114572543455208e-15);  // 1/19!, -1/17!
        S = horner(q, S, 7.6471637318198164e-13);                      // 1/15!
        S = horner(q, S, -1.6059043836821613e-10);                     // -1/13!
        S = horner(q, S, 2.5052108385441719e-8);                       // 1/11!
        S = horner(q, S, -2.7557319223985891e-6);                      // -1/9!
        S = horner(q, S, 1.9841269841269841e-4);                       // 1/7!
        S = horner(q, S, -8.3333333333333333e-3);                      // -1/5!
        S = horner(q, S, 1.6666666666666667e-1);                       // 1/3!
        S = fma(-q, S, 1.0);
        C = horner_first(q, 4.1103176233121648e-19, -1.5619206968586226e-16);  // 1/20!, -1/18!
        C = horner(q, C, 4.7794773323873853e-14);                      // 1/16!
        C = horner(q, C, -1.1470745597729725e-11);                     // -1/14!
        C = horner(q, C, 2.0876756987868099e-9);                       // 1/12!
        C = horner(q, C, -2.7557319223985891e-7);                      // -1/10!
        C = horner(q, C, 2.4801587301587302e-5);                       // 1/8!
        C = horner(q, C, -1.3888888888888889e-3);                      // -1/6!
        C = horner(q, C, 4.1666666666666667e-2);                       // 1/4!
        C = fma(-q, C, 0.5);
    }
    // Terms k = 0 .. 5 only: for q <= 1/16 the first dropped ones,
    // q^6 / 13! and q^6 / 14!, are below 1e-17 relative.
    static __device__ __forceinline__ void coeffs_short(double q, double &S, double &C) {
        S = horner_first(q, 2.5052108385441719e-8, -2.7557319223985891e-6);  // 1/11!, -1/9!
        S = horner(q, S, 1.9841269841269841e-4);                         // 1/7!
        S = horner(q, S, -8.3333333333333333e-3);                        // -1/5!
        S = horner(q, S, 1.6666666666666667e-1);                         // 1/3!
        S = fma(-q, S, 1.0);
        C = horner_first(q, 2.0876756987868099e-9, -2.7557319223985891e-7);  // 1/12!, -1/10!
        C = horner(q, C, 2.4801587301587302e-5);                         // 1/8!
        C = horner(q, C, -1.3888888888888889e-3);                        // -1/6!
        C = horner(q, C, 4.1666666666666667e-2);                         // 1/4!
        C = fma(-q, C, 0.5);
    }
    static __device__ __forceinline__ void big(double B2, double gdt, double &a, double &b) {
        const double nb = sqrt(B2);
        double sh, ch;
        sincos(0.5 * gdt * nb, &sh, &ch);
        a = -2.0 * sh * ch / nb;
        b = 2.0 * sh * sh / B2;
    }
};

__device__ __forceinline__ void rot_coeffs(double B2, double gdt, double k2, double &a, double &b) {
    const double q = k2 * B2;
    if (q <= 0.0625) {  // rotations under a quarter radian: most raster steps
        double S, C;
        Series::coeffs_short(q, S, C);
        a = -gdt * S;
        b = k2 * C;
    } else if (q <= 1.0) {
        double S, C;
        Series::coeffs(q, S, C);
        a = -gdt * S;
        b = k2 * C;
    } else {
        Series::big(B2, gdt, a, b);
    }
}

}  // namespace gbs
