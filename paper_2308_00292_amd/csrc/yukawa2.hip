// Tables of the 2-D kernel K_0(lambda r) (Sec. 4.6, eq. yukawaPSWFkernels,
// taken with the transform 2 pi/(k^2 + lambda^2) of K_0(lambda r)).
//
// The split is not scale invariant: everything depends on mu = lambda S_b s_l
// (lambda S_b the problem's scaled parameter, s_l = 2^-l), so the plan holds
// one table per (problem, level), index b * nlevels + l:
//  * D_l weights (h_l/2pi)^2 Dhat_l(h_l |m|), h_l s_l = 2 pi/3:
//      w(m) = 2 pi [psi(rho/(2c)) - psi(rho/c)] / (9 psi(0) rho^2),
//      rho = sqrt((2 pi |m|/3)^2 + mu^2)                           (host);
//  * the smooth part of the residual R_l(r) = K_0(lambda S_b r) - M_l(r),
//      M_l(x s_l) = int_0^T psi(sqrt(t^2 + mu^2)/c)/psi(0) J_0(t x) t/(t^2 + mu^2) dt,
//      T = sqrt(4c^2 - mu^2) (the mollifier beyond argument 2 is dropped),
//    as a Chebyshev series in u = 2x^2 - 1, and M_l(0) for the r = 0 term.
//    The quadratures (49 per table: 48 Chebyshev nodes and x = 0) run on the
//    device, one workgroup each: composite Gauss-Legendre on panels doubling
//    in length towards T, J_0 by the trapezoidal rule on Bessel's integral
//    J_0(z) = (1/pi) int_0^pi cos(z sin th) dth (exponentially convergent for
//    this periodic analytic integrand), psi(x)/psi(0) on [0,2] from a
//    piecewise Chebyshev interpolant built on the host;
//  * the root's windowed kernel per problem (Sec. 4.7): psi(kappa/c)/psi(0)
//    times the transform of K_0 truncated at A = 1 + sqrt 2,
//      That(k) = 2 pi {1 + A [k J_1(kA) K_0(lA) - l J_0(kA) K_1(lA)]}/(k^2 + l^2)  (host).
#include <algorithm>
#include <cmath>

#include "dmk_internal.h"

namespace dmk {

namespace {

constexpr int TPB = 256;
constexpr int YNODES = 48;          // Chebyshev nodes of the residual tables
constexpr int PS_PAN = 32;          // psi interpolant: panels on [0, 2]
constexpr int PS_DEG = 16;
constexpr int Q_GL = 16, Q_PAN = 44;  // quadrature: 16-point rule on 44 panels
constexpr int J0_N = 48;             // trapezoidal points of Bessel's integral (z <= 2c < 36)

__device__ inline double psi_interp(const double *pc, double x)
{
    // x in [0, 2]
    int k = (int)(x * (PS_PAN / 2.0));
    k = k < 0 ? 0 : (k >= PS_PAN ? PS_PAN - 1 : k);
    const double a = 2.0 * k / PS_PAN, h = 2.0 / PS_PAN;
    const double u = 2.0 * (x - a) / h - 1.0;
    const double *c = pc + k * (PS_DEG + 1);
    double b1 = 0.0, b2 = 0.0;
    for (int j = PS_DEG; j >= 1; --j) {
        double b0 = c[j] + 2.0 * u * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + u * b1 - b2;
}

// One block per (table, node): M_l at x_j (j < YNODES) or at x = 0.
__global__ void __launch_bounds__(TPB) k_ytab(const double *lam_b, int nlev, double c, const double *pc,
                                              const double *glx, const double *glw, double *out)
{
    __shared__ double sn[J0_N];
    __shared__ double red[TPB];
    const int tab = blockIdx.x / (YNODES + 1), j = blockIdx.x % (YNODES + 1);
    const int b = tab / nlev, l = tab % nlev;
    const double mu = lam_b[b] * ldexp(1.0, -l);
    for (int i = threadIdx.x; i < J0_N; i += TPB) sn[i] = sin(M_PI * i / J0_N);
    __syncthreads();
    const double T2 = 4.0 * c * c - mu * mu;
    double x = 0.0;
    if (j < YNODES) {
        const double u = cos(M_PI * (j + 0.5) / YNODES);
        x = sqrt(0.5 * (u + 1.0));
    }
    double acc = 0.0;
    if (T2 > 0.0) {
        const double T = sqrt(T2);
        for (int k = threadIdx.x; k < Q_GL * Q_PAN; k += TPB) {
            const int pnl = k / Q_GL, q = k % Q_GL;
            const double a = (pnl == 0) ? 0.0 : T * ldexp(1.0, pnl - Q_PAN);
            const double e = T * ldexp(1.0, pnl + 1 - Q_PAN);
            const double t = 0.5 * (a + e) + 0.5 * (e - a) * glx[q];
            const double w = 0.5 * (e - a) * glw[q];
            const double kap2 = t * t + mu * mu;
            double arg = sqrt(kap2) / c;
            arg = arg > 2.0 ? 2.0 : arg;
            const double g = psi_interp(pc, arg) * t / kap2;
            const double z = t * x;
            double j0 = 0.0;
            for (int i = 0; i < J0_N; ++i) j0 += cos(z * sn[i]);
            acc += w * g * (j0 / J0_N);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// psi(x)/psi(0) on [0, xmax] as piecewise Chebyshev series of degree PS_DEG
// on panels of width 2/PS_PAN (host and device use the same coefficients).
std::vector<double> psi_panels(const Tables &t, int npan)
{
    std::vector<double> pc((size_t)npan * (PS_DEG + 1));
    const int M = PS_DEG + 1;
    const double h = 2.0 / PS_PAN;
    for (int k = 0; k < npan; ++k) {
        std::vector<double> f(M);
        for (int i = 0; i < M; ++i) {
            double u = std::cos(M_PI * (i + 0.5) / M);
            f[i] = pswf_eval(t, k * h + 0.5 * h * (u + 1.0)) / t.psi0;
        }
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int i = 0; i < M; ++i) s += f[i] * std::cos(M_PI * j * (i + 0.5) / M);
            pc[(size_t)k * M + j] = (j == 0 ? 1.0 : 2.0) * s / M;
        }
    }
    return pc;
}

double psi_host(const Tables &t, const std::vector<double> &pc, int npan, double x)
{
    x = std::fabs(x);
    const double h = 2.0 / PS_PAN;
    int k = (int)(x / h);
    if (k >= npan) return pswf_eval(t, x) / t.psi0;
    const double u = 2.0 * (x - k * h) / h - 1.0;
    const double *c = pc.data() + (size_t)k * (PS_DEG + 1);
    double b1 = 0.0, b2 = 0.0;
    for (int j = PS_DEG; j >= 1; --j) {
        double b0 = c[j] + 2.0 * u * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + u * b1 - b2;
}

}  // namespace

void build_yukawa_tables(Plan *P, hipStream_t s)
{
    const Tables &t = P->tab;
    const int nprob = P->nprob, L = P->nlevels;
    const int64_t ntab = (int64_t)nprob * L;
    const double c = t.prm.c;
    // scaled parameters lambda S_b
    std::vector<double> lam(nprob);
    for (int b = 0; b < nprob; ++b) lam[b] = P->lambda * P->pside[b];
    // psi interpolant: [0, 2] for the device, [0, 8] for the host weights
    const int npan_host = 4 * PS_PAN;
    std::vector<double> pc_host = psi_panels(t, npan_host);
    std::vector<double> pc_dev(pc_host.begin(), pc_host.begin() + (size_t)PS_PAN * (PS_DEG + 1));

    // ---- D_l weights per table, half spectrum [m1][m2 >= 0]
    const int nf = t.nf, nn = t.nn, nh = t.nh;
    const int64_t nm = (int64_t)nn * nh;
    std::vector<double> wd((size_t)ntab * nm);
    {
        const int maxk2 = 2 * nf * nf;
        std::vector<double> memo(maxk2 + 1);
        for (int64_t tb = 0; tb < ntab; ++tb) {
            const double mu = lam[tb / L] * std::ldexp(1.0, -(int)(tb % L));
            for (int k2 = 0; k2 <= maxk2; ++k2) {
                const double rho2 = 4.0 * M_PI * M_PI * k2 / 9.0 + mu * mu, rho = std::sqrt(rho2);
                memo[k2] = 2.0 * M_PI *
                           (psi_host(t, pc_host, npan_host, rho / (2.0 * c)) - psi_host(t, pc_host, npan_host, rho / c)) /
                           (9.0 * rho2);
            }
            double *w = wd.data() + tb * nm;
            for (int m1 = -nf; m1 <= nf; ++m1)
                for (int m2 = 0; m2 <= nf; ++m2) w[(m1 + nf) * nh + m2] = memo[m1 * m1 + m2 * m2];
        }
    }
    // ---- root W_0 weights per problem
    const int nw = t.nw, nwn = t.nwn, nwh = t.nwh;
    std::vector<double> ww((size_t)nprob * nwn * nwh);
    {
        const double Atr = 1.0 + std::sqrt(2.0), h = t.prm.hw, fac = std::pow(h / (2.0 * M_PI), 2);
        const int maxk2 = 2 * nw * nw;
        std::vector<double> memo(maxk2 + 1);
        for (int b = 0; b < nprob; ++b) {
            const double l = lam[b];
            const double k0A = std::cyl_bessel_k(0.0, l * Atr), k1A = std::cyl_bessel_k(1.0, l * Atr);
            for (int k2 = 0; k2 <= maxk2; ++k2) {
                const double k = h * std::sqrt((double)k2);
                const double That = 2.0 * M_PI *
                                    (1.0 + Atr * (k * std::cyl_bessel_j(1.0, k * Atr) * k0A -
                                                  l * std::cyl_bessel_j(0.0, k * Atr) * k1A)) /
                                    (k * k + l * l);
                memo[k2] = fac * That * psi_host(t, pc_host, npan_host, std::sqrt(k * k + l * l) / c);
            }
            double *w = ww.data() + (size_t)b * nwn * nwh;
            for (int m1 = -nw; m1 <= nw; ++m1)
                for (int m2 = 0; m2 <= nw; ++m2) w[(m1 + nw) * nwh + m2] = memo[m1 * m1 + m2 * m2];
        }
    }
    // ---- residual smooth parts: quadratures on the device, series on the host
    std::vector<double> vals((size_t)ntab * (YNODES + 1));
    {
        std::vector<double> glx(Q_GL), glw(Q_GL);
        for (int i = 0; i < Q_GL; ++i) {  // Newton on P_Q_GL
            double z = std::cos(M_PI * (i + 0.75) / (Q_GL + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= Q_GL; ++k) {
                    double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = pk;
                }
                dp = Q_GL * (z * p1 - p0) / (z * z - 1.0);
                double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= Q_GL; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = Q_GL * (z * p1 - p0) / (z * z - 1.0);
            glx[i] = z;
            glw[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
        double *d_lam = (double *)dalloc(P, nprob * sizeof(double));
        double *d_pc = nullptr, *d_gl = nullptr, *d_out = nullptr;
        DMK_HIP(hipMalloc(&d_pc, pc_dev.size() * sizeof(double)));
        DMK_HIP(hipMalloc(&d_gl, 2 * Q_GL * sizeof(double)));
        DMK_HIP(hipMalloc(&d_out, vals.size() * sizeof(double)));
        try {
            DMK_HIP(hipMemcpyAsync(d_lam, lam.data(), nprob * sizeof(double), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(d_pc, pc_dev.data(), pc_dev.size() * sizeof(double), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(d_gl, glx.data(), Q_GL * sizeof(double), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(d_gl + Q_GL, glw.data(), Q_GL * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_ytab, dim3((unsigned)(ntab * (YNODES + 1))), dim3(TPB), 0, s, d_lam, L, c, d_pc,
                               d_gl, d_gl + Q_GL, d_out);
            DMK_HIP(hipGetLastError());
            DMK_HIP(hipMemcpyAsync(vals.data(), d_out, vals.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipFree(d_pc);
            (void)hipFree(d_gl);
            (void)hipFree(d_out);
            throw;
        }
        (void)hipFree(d_pc);
        (void)hipFree(d_gl);
        (void)hipFree(d_out);
        P->y_lam = d_lam;
    }
    std::vector<double> cheb((size_t)ntab * YNODES), self(ntab);
    int deg = 0, deg32 = 0;
    for (int64_t tb = 0; tb < ntab; ++tb) {
        const double *f = vals.data() + tb * (YNODES + 1);
        double *cf = cheb.data() + tb * YNODES;
        double cmax = 0.0;
        for (int j = 0; j < YNODES; ++j) {
            double sum = 0.0;
            for (int k = 0; k < YNODES; ++k) sum += f[k] * std::cos(M_PI * j * (k + 0.5) / YNODES);
            cf[j] = (j == 0 ? 1.0 : 2.0) * sum / YNODES;
            cmax = std::max(cmax, std::fabs(cf[j]));
        }
        self[tb] = f[YNODES];
        int d = YNODES - 1, d32;
        while (d > 0 && std::fabs(cf[d]) < 1e-15 * cmax) d--;
        d32 = d;
        while (d32 > 0 && std::fabs(cf[d32]) < 1e-8 * cmax) d32--;
        deg = std::max(deg, d);
        deg32 = std::max(deg32, d32);
    }
    P->y_deg = deg;
    P->y_deg32 = deg32;
    auto up = [&](const std::vector<double> &v) {
        double *d = (double *)dalloc(P, std::max<size_t>(v.size(), 1) * sizeof(double));
        DMK_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
        return d;
    };
    std::vector<std::vector<float>> keep;
    auto upf = [&](const std::vector<double> &v) {
        keep.emplace_back(v.begin(), v.end());
        float *d = (float *)dalloc(P, std::max<size_t>(v.size(), 1) * sizeof(float));
        DMK_HIP(hipMemcpyAsync(d, keep.back().data(), v.size() * sizeof(float), hipMemcpyHostToDevice, s));
        return d;
    };
    P->y_wd64 = up(wd);
    P->y_wd32 = upf(wd);
    P->y_ww = up(ww);
    P->y_cheb64 = up(cheb);
    P->y_cheb32 = upf(cheb);
    P->y_self = up(self);
    DMK_HIP(hipStreamSynchronize(s));
}

}  // namespace dmk
