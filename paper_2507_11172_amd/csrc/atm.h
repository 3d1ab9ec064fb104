// Axilrod-Teller-Muto three-body term (Sec. 2.1) in the squared edge lengths of a triangle,
// shared by the cutoff and the DirectSum triplet kernels.
#pragma once

#include "common.h"

namespace mts {

// 1/sqrt(x): hardware estimate refined by two Newton-Raphson steps y <- y (3 - x y^2)/2
// (quadratic convergence from the ~2^-22 estimate to below one FP64 ulp of error).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt_nr(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// ATM potential in squared edge lengths a = |u|^2, b = |w|^2, c = |v|^2 (u: i->j, w: i->k,
// v: j->k).  By the law of cosines the cosine product of Sec. 2.1 is t1 t2 t3 / (8abc),
// t1 = a+b-c, t2 = a-b+c, t3 = b+c-a, so
//   phi = nu [P^-3/2 + 3/8 T P^-5/2],  P = abc,  T = t1 t2 t3.
// Returns phi and g_a = 2 dphi/da, g_b, g_c; the forces are
//   F_i = g_a u + g_b w,  F_j = -g_a u + g_c v,  F_k = -g_b w - g_c v,
// and the triplet's virial sum_x x.F = u.F_j + w.F_k = -(a g_a + b g_b + c g_c).
// Arranged for few operations: the edge products are shared, the factor 2 nu is folded
// into the coefficients (q2 = 2 nu 3/8 P^-5/2, kp = 2 nu K / P with
// K = -3/2 P^-3/2 - 15/16 T P^-5/2), and t1..t3 come from s = a + b + c.
template <typename T>
__device__ __forceinline__ void atm_terms(T a, T b, T c, T nu, T &phi, T &ga, T &gb, T &gc) {
    const T ab = a * b, bc = b * c, ac = a * c;
    const T P = ab * c;
    const T rs = rsqrt_t<T>(P);         // P^-1/2
    const T ip = rs * rs;               // P^-1
    const T p32 = rs * ip;              // P^-3/2
    const T p52 = p32 * ip;             // P^-5/2
    const T sum = (a + b) + c;
    const T t1 = fma(T(-2), c, sum), t2 = fma(T(-2), b, sum), t3 = fma(T(-2), a, sum);
    const T t12 = t1 * t2;
    const T tt = t12 * t3;
    const T q2 = (T(0.75) * nu) * p52;
    const T kp = fma((T(-1.875) * nu) * tt, p52, (T(-3) * nu) * p32) * ip;
    ga = fma(kp, bc, q2 * fma(a + a, t3, -t12));
    gb = fma(kp, ac, q2 * fma(b + b, t2, -(t1 * t3)));
    gc = fma(kp, ab, q2 * fma(c + c, t1, -(t2 * t3)));
    phi = fma(T(0.5) * q2, tt, nu * p32);
}

}  // namespace mts
