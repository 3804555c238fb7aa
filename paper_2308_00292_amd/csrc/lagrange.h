// Lagrange basis of the Chebyshev proxy nodes at a point, with one division.
#pragma once

#include <hip/hip_runtime.h>

namespace dmk {

// Lagrange basis of the nodes at xi with one division (prefix products of
// the differences, Montgomery's batch inversion), barycentric weights bw.
template <typename T, int P>
__device__ inline void lagrange_row_fast(const T *xc, const T *bw, T xi, T (&out)[P])
{
    T d[P], pre[P];
    int hit = -1;
#pragma unroll
    for (int a = 0; a < P; ++a) {
        d[a] = xi - xc[a];
        if (d[a] == T(0)) hit = a;
    }
    if (hit >= 0) {
#pragma unroll
        for (int a = 0; a < P; ++a) out[a] = (a == hit) ? T(1) : T(0);
        return;
    }
    pre[0] = d[0];
#pragma unroll
    for (int a = 1; a < P; ++a) pre[a] = pre[a - 1] * d[a];
    T inv = T(1) / pre[P - 1];
    T den = T(0);
#pragma unroll
    for (int a = P - 1; a >= 1; --a) {
        out[a] = bw[a] * (inv * pre[a - 1]);
        inv *= d[a];
        den += out[a];
    }
    out[0] = bw[0] * inv;
    den += out[0];
    const T r = T(1) / den;
#pragma unroll
    for (int a = 0; a < P; ++a) out[a] *= r;
}

}  // namespace dmk
