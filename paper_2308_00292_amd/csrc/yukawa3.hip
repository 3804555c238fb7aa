// Tables of the 3-D kernel e^{-lambda r}/(4 pi r) (Sec. 4.6, eq.
// yukawaPSWFkernels with the transform 4 pi/(k^2 + lambda^2) of
// e^{-lambda r}/r; the 1/(4 pi) joins the unit change in k_finalize).
//
// The split is not scale invariant: with lambda' = lambda S (root-box units)
// everything depends on mu_l = lambda' s_l, so the plan holds one table per
// level l:
//  * D_l weights (h_l/2pi)^3 Dhat_l(h_l |m|), h_l s_l = 2 pi/3, in the
//    half-spectrum layout [m1][m3 >= 0][m2] of the translation:
//      w(m) = 4 pi [psi(rho/(2c)) - psi(rho/c)] / (27 s_l psi(0) rho^2),
//      rho^2 = (2 pi |m|/3)^2 + mu_l^2;
//  * the mollified kernel M_l = K * G_l (Ghat_l = psi(kappa s_l/c)/psi(0)),
//      M_l(x s_l) = m_l(x)/s_l,
//      m_l(x) = (2/pi) int_0^T psi(sqrt(t^2+mu^2)/c)/psi(0) t sin(t x)/(x (t^2 + mu^2)) dt,
//      T = sqrt(4c^2 - mu^2) (the mollifier beyond argument 2 is dropped),
//    as a Chebyshev series in u = 2x^2 - 1 (48 nodes), and M_l(0); the
//    residual of a pair is e^{-lambda' r}/r - M_l(r) for r < s_l;
//  * the root's windowed kernel (Sec. 4.7): psi(kappa/c)/psi(0) times the
//    transform of the kernel cut at A = 1 + sqrt 3,
//      That(k) = 4 pi [k - e^{-lambda' A}(lambda' sin kA + k cos kA)]/(k (k^2 + lambda'^2)),
//      That(0) = 4 pi [1 - e^{-lambda' A}(1 + lambda' A)]/lambda'^2,
//    in the [m3 >= 0][m2][m1] layout of the root stage.
// All on the host, once per plan (at most 21 levels).
#include <algorithm>
#include <cmath>

#include "dmk_internal.h"

namespace dmk {

namespace {

constexpr int YN = 48;                // Chebyshev nodes of the mollified-kernel tables
constexpr int QG = 16, QPAN = 48;     // quadrature: 16-point Gauss-Legendre panels, geometric towards 0

void gauss_legendre_nodes(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// 1 - e^{-x}(1 + x) without cancellation at small x
double one_minus_exp_poly(double x)
{
    if (x >= 0.5) return 1.0 - std::exp(-x) * (1.0 + x);
    // x^2/2 - 2 x^3/3! + 3 x^4/4! - ...
    double term = 0.5 * x * x, f = 0.0;
    for (int k = 2; k < 40; ++k) {
        f += (k - 1) * term;
        term *= -x / (k + 1);
    }
    return f;
}

}  // namespace

void build_yukawa3_tables(Plan *P, hipStream_t s)
{
    const Tables &t = P->tab;
    const int L = P->nlevels;
    const double c = t.prm.c, lam = P->lambda * P->pside[0];
    auto psi = [&](double x) { return pswf_eval(t, x) / t.psi0; };

    // ---- D_l weights per level, layout [m1][m3][m2]
    const int nf = t.nf, nn = t.nn, nh = t.nh;
    const int64_t nm = (int64_t)nh * nn * nn;
    std::vector<double> wd((size_t)L * nm);
    {
        const int maxk2 = 3 * nf * nf;
        std::vector<double> memo(maxk2 + 1);
        for (int l = 0; l < L; ++l) {
            const double sl = std::ldexp(1.0, -l), mu = lam * sl;
            for (int k2 = 0; k2 <= maxk2; ++k2) {
                const double rho2 = 4.0 * M_PI * M_PI * k2 / 9.0 + mu * mu, rho = std::sqrt(rho2);
                memo[k2] = 4.0 * M_PI * (psi(rho / (2.0 * c)) - psi(rho / c)) / (27.0 * sl * rho2);
            }
            double *w = wd.data() + (size_t)l * nm;
            for (int m1 = -nf; m1 <= nf; ++m1)
                for (int m3 = 0; m3 <= nf; ++m3)
                    for (int m2 = -nf; m2 <= nf; ++m2)
                        w[((size_t)(m1 + nf) * nh + m3) * nn + (m2 + nf)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
        }
    }
    // ---- root W_0 weights, layout [m3][m2][m1]
    const int nw = t.nw, nwn = t.nwn, nwh = t.nwh;
    std::vector<double> ww((size_t)nwh * nwn * nwn);
    {
        const double A = 1.0 + std::sqrt(3.0), h = t.prm.hw, fac = std::pow(h / (2.0 * M_PI), 3);
        const double ea = std::exp(-lam * A);
        const int maxk2 = 3 * nw * nw;
        std::vector<double> memo(maxk2 + 1);
        for (int k2 = 0; k2 <= maxk2; ++k2) {
            const double k = h * std::sqrt((double)k2);
            const double That = (k2 == 0) ? 4.0 * M_PI * one_minus_exp_poly(lam * A) / (lam * lam)
                                          : 4.0 * M_PI * (k - ea * (lam * std::sin(k * A) + k * std::cos(k * A))) /
                                                (k * (k * k + lam * lam));
            memo[k2] = fac * That * psi(std::sqrt(k * k + lam * lam) / c);
        }
        for (int m3 = 0; m3 <= nw; ++m3)
            for (int m2 = -nw; m2 <= nw; ++m2)
                for (int m1 = -nw; m1 <= nw; ++m1)
                    ww[((size_t)m3 * nwn + (m2 + nw)) * nwn + (m1 + nw)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
    // ---- mollified kernel per level: values at the Chebyshev nodes and at 0
    std::vector<double> cheb((size_t)L * YN), self(L);
    int deg = 0, deg32 = 0;
    {
        std::vector<double> gx, gw;
        gauss_legendre_nodes(QG, gx, gw);
        std::vector<double> tq, wq, f(YN);
        for (int l = 0; l < L; ++l) {
            const double sl = std::ldexp(1.0, -l), mu = lam * sl, T2 = 4.0 * c * c - mu * mu;
            tq.clear();
            wq.clear();
            if (T2 > 0.0) {
                const double T = std::sqrt(T2);
                // panels [T 2^-k-1, T 2^-k] for k < QPAN - 1, then [0, T 2^-(QPAN-1)]
                for (int k = 0; k < QPAN; ++k) {
                    const double b = std::ldexp(T, -k), a = (k == QPAN - 1) ? 0.0 : 0.5 * b;
                    for (int q = 0; q < QG; ++q) {
                        const double tt = 0.5 * (a + b) + 0.5 * (b - a) * gx[q];
                        const double kap2 = tt * tt + mu * mu;
                        tq.push_back(tt);
                        wq.push_back(0.5 * (b - a) * gw[q] * (2.0 / M_PI) * psi(std::sqrt(kap2) / c) * tt / kap2);
                    }
                }
            }
            for (int j = 0; j < YN; ++j) {
                const double u = std::cos(M_PI * (j + 0.5) / YN), x = std::sqrt(0.5 * (u + 1.0));
                double acc = 0.0;
                for (size_t k = 0; k < tq.size(); ++k) acc += wq[k] * std::sin(tq[k] * x) / x;
                f[j] = acc;
            }
            double a0 = 0.0;
            for (size_t k = 0; k < tq.size(); ++k) a0 += wq[k] * tq[k];
            self[l] = a0 / sl;
            double *cf = cheb.data() + (size_t)l * YN, cmax = 0.0;
            for (int j = 0; j < YN; ++j) {
                double acc = 0.0;
                for (int k = 0; k < YN; ++k) acc += f[k] * std::cos(M_PI * j * (k + 0.5) / YN);
                cf[j] = (j == 0 ? 1.0 : 2.0) * acc / YN;
                cmax = std::max(cmax, std::fabs(cf[j]));
            }
            int d = YN - 1;
            while (d > 0 && std::fabs(cf[d]) < 1e-15 * cmax) d--;
            int d32 = d;
            while (d32 > 0 && std::fabs(cf[d32]) < 1e-8 * cmax) d32--;
            deg = std::max(deg, d);
            deg32 = std::max(deg32, d32);
        }
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
    P->d_ww = P->y_ww;  // the root stage applies the Yukawa window
    P->y_cheb64 = up(cheb);
    P->y_cheb32 = upf(cheb);
    P->y_self = up(self);
    P->y_lam = up(std::vector<double>(1, lam));
    DMK_HIP(hipStreamSynchronize(s));
}

}  // namespace dmk
