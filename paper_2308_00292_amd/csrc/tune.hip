// Direct sums at sampled targets, for the autotuner's accuracy gate: the
// potential of the caller's charges by the definition u_i = sum_{j != i,
// r_ij > 0} K(r_ij) q_j (within target i's own problem), in FP64 with
// compensated accumulation.  One block per target.
#include <cmath>

#include "dmk_internal.h"
#include "kfun.h"

namespace dmk {

namespace {

constexpr int TT = 256;

__device__ inline double kernel_value(int dim, int kernel, double lam, double r)
{
    if (dim == 3) {
        if (kernel == DMK_POWER2) return 1.0 / (r * r);
        const double k = 1.0 / (4.0 * M_PI * r);
        return (kernel == DMK_YUKAWA) ? k * exp(-lam * r) : k;
    }
    if (kernel == DMK_YUKAWA) return bessel_k0<double>(lam * r);
    return -log(r) / (2.0 * M_PI);
}

__global__ void __launch_bounds__(TT) k_direct_sample(int dim, int kernel, double lam, const double *pts,
                                                      const double *q, const int64_t *off, int nprob,
                                                      const int64_t *tidx, double *out)
{
    __shared__ double red[TT];
    const int64_t i = tidx[blockIdx.x];
    int lo = 0, hi = nprob - 1;  // the problem b with off[b] <= i < off[b+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const double xi = pts[dim * i], yi = pts[dim * i + 1], zi = (dim == 3) ? pts[dim * i + 2] : 0.0;
    double s = 0.0, c = 0.0;  // Kahan-Babuska
    for (int64_t j = off[lo] + threadIdx.x; j < off[lo + 1]; j += TT) {
        if (j == i) continue;
        const double dx = xi - pts[dim * j], dy = yi - pts[dim * j + 1], dz = (dim == 3) ? zi - pts[dim * j + 2] : 0.0;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) continue;
        const double v = kernel_value(dim, kernel, lam, r) * q[j];
        const double t = s + v;
        c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    red[threadIdx.x] = s + c;
    __syncthreads();
    for (int w = TT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

void direct_sample(int dim, int kernel, double lam, const double *pts, const double *q, const int64_t *d_off,
                   int nprob, const int64_t *d_tidx, int ntgt, double *d_out, hipStream_t s)
{
    if (ntgt <= 0) return;
    hipLaunchKernelGGL(k_direct_sample, dim3((unsigned)ntgt), dim3(TT), 0, s, dim, kernel, lam, pts, q, d_off, nprob,
                       d_tidx, d_out);
    DMK_HIP(hipGetLastError());
}

}  // namespace dmk
