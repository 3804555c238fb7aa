// Device functions of the kernels shared by several translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace dmk {

// ------------------------------------------------------------ K_0(z), z > 0
// z <= 2: the ascending series -(log(z/2) + gamma) I_0(z) + sum_k (z^2/4)^k H_k/(k!)^2
// (Abramowitz & Stegun 9.6.13); z > 2: K_0(z) = int_0^inf exp(-z cosh t) dt by
// the trapezoidal rule (geometric convergence for this analytic integrand).
template <typename T>
__device__ inline T bessel_k0(T z)
{
    if (z <= T(2)) {
        const T y = T(0.25) * z * z;
        T term = T(1), i0 = T(1), sum = T(0), H = T(0);
        for (int k = 1; k <= 14; ++k) {
            term *= y / T(k * k);
            H += T(1) / T(k);
            i0 += term;
            sum += term * H;
        }
        return -(log(T(0.5) * z) + T(0.57721566490153286061)) * i0 + sum;
    }
    const T h = T(0.125);
    const T cut = sizeof(T) == 8 ? T(700) : T(87);
    T s = T(0.5) * exp(-z);
    for (int j = 1; j < 200; ++j) {
        const T ch = cosh(T(j) * h);
        if (z * ch > cut) break;
        s += exp(-z * ch);
    }
    return h * s;
}

}  // namespace dmk
