/*
 * yuk3.c -- the 3-D Yukawa kernel K(r) = e^{-lambda r}/(4 pi r) split in
 * Fourier space with the PSWF (Sec. 4.6, eq. yukawaPSWFkernels) and its
 * windowed root kernel (Sec. 4.7, truncated-kernel window).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Internally K(r) = e^{-lambda r}/r (the factor 1/(4 pi) is applied with the
 * unit change at the end, as for 1/r), whose 3-D transform is
 * 4 pi/(k^2 + lambda^2).  With kappa^2 = k^2 + lambda^2 and box side s_l:
 *   mollifier  Ghat_l(k) = psi(kappa s_l/c)/psi(0);
 *   Dhat_l(k)  = 4 pi [psi(kappa s_{l+1}/c) - psi(kappa s_l/c)]/(psi(0) kappa^2);
 *   M_l        = K * G_l, the mollified kernel, whose radial inverse
 *                transform is M_l(r) = (2/(pi r)) int_0^inf k sin(kr) Ghat_l(k)/kappa^2 dk;
 *                in x = r/s_l and mu = lambda s_l: M_l(r) = m_mu(x)/s_l with
 *                m_mu(x) = (2/pi) int_0^T t (sin(t x)/x) psi(sqrt(t^2+mu^2)/c)/(psi(0)(t^2+mu^2)) dt,
 *                T^2 = 4c^2 - mu^2 (the mollifier beyond argument 2 is below 1e-9
 *                of psi(0) and is dropped);
 *   residual   R_l(r) = K(r) - M_l(r) for r < s_l, 0 beyond;
 *   root       What_0(k) = Ghat_0(k) That(k), That the transform of K cut at
 *                A = (1 + sqrt 3) s_0:
 *                That(k) = (4 pi/k) int_0^A e^{-lambda r} sin(kr) dr
 *                        = 4 pi [k - e^{-lambda A}(lambda sin kA + k cos kA)]/(k (k^2 + lambda^2)),
 *                That(0) = 4 pi [1 - e^{-lambda A}(1 + lambda A)]/lambda^2.
 * All lambdas here are in root-box units (lambda S); the oracle requires
 * 1e-3 <= lambda S (below that the k -> 0 differences of psi lose digits
 * and the kernel is 1/r to that precision anyway).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static double side(int l) { return ldexp(1.0, -l); }

double orc_y3_dhat(const orc_pswf *ps, double lam, int l, double k)
{
    const double kap2 = k * k + lam * lam, kap = sqrt(kap2);
    return 4.0 * M_PI *
           (orc_pswf_eval_ext(ps, kap * side(l + 1) / ps->c) - orc_pswf_eval_ext(ps, kap * side(l) / ps->c)) /
           (ps->psi0 * kap2);
}

double orc_y3_that(double lam, double k)
{
    const double A = 1.0 + sqrt(3.0);
    const double ea = exp(-lam * A);
    if (k == 0.0) {
        /* 1 - e^{-x}(1 + x) = sum_{n>=2} (-1)^n (n-1) x^n/n!, summed directly for small x */
        const double x = lam * A;
        double f;
        if (x < 0.5) {
            double term = x * x / 2.0;
            f = 0.0;
            for (int nn = 2; nn < 40; ++nn) {
                f += (nn - 1) * term;
                term *= -x / (nn + 1);
            }
        } else {
            f = 1.0 - ea * (1.0 + x);
        }
        return 4.0 * M_PI * f / (lam * lam);
    }
    return 4.0 * M_PI * (k - ea * (lam * sin(k * A) + k * cos(k * A))) / (k * (k * k + lam * lam));
}

double orc_y3_w0hat(const orc_pswf *ps, double lam, double k)
{
    const double kap = sqrt(k * k + lam * lam);
    return orc_pswf_eval_ext(ps, kap * side(0) / ps->c) / ps->psi0 * orc_y3_that(lam, k);
}

/* ------------------------------------------- mollified kernel by quadrature */
#define Y3_NGL 24
#define Y3_NPANEL 44

/* Gauss-Legendre panels on [0, T]: a first panel [0, T 2^{1-NPANEL}], then
 * panels doubling in length up to T; w includes the smooth weight function
 * (2/pi) t psi(sqrt(t^2+mu^2)/c)/(psi(0)(t^2+mu^2)).  Returns the node count
 * (0 when the mollifier vanishes everywhere, mu >= 2c). */
static int y3_nodes(const orc_pswf *ps, double mu, double *t, double *w)
{
    const double c = ps->c, T2 = 4.0 * c * c - mu * mu;
    if (T2 <= 0.0) return 0;
    const double T = sqrt(T2);
    double gx[Y3_NGL], gw[Y3_NGL];
    orc_gauss_legendre(Y3_NGL, gx, gw);
    int k = 0;
    for (int pnl = 0; pnl < Y3_NPANEL; ++pnl) {
        double a = (pnl == 0) ? 0.0 : T * ldexp(1.0, pnl - Y3_NPANEL);
        double b = T * ldexp(1.0, pnl + 1 - Y3_NPANEL);
        for (int q = 0; q < Y3_NGL; ++q, ++k) {
            t[k] = 0.5 * (a + b) + 0.5 * (b - a) * gx[q];
            const double kap2 = t[k] * t[k] + mu * mu;
            w[k] = 0.5 * (b - a) * gw[q] * (2.0 / M_PI) * t[k] * orc_pswf_eval_ext(ps, sqrt(kap2) / c) /
                   (ps->psi0 * kap2);
        }
    }
    return k;
}

/* sin(t x)/x, with its limit t at x = 0 */
static double sinc_t(double t, double x) { return (x == 0.0) ? t : sin(t * x) / x; }

double orc_y3_smooth_quad(const orc_pswf *ps, double mu, double x)
{
    double t[Y3_NGL * Y3_NPANEL], w[Y3_NGL * Y3_NPANEL];
    const int nq = y3_nodes(ps, mu, t, w);
    double s = 0.0;
    for (int k = 0; k < nq; ++k) s += w[k] * sinc_t(t[k], x);
    return s;
}

int orc_y3_split_init(const orc_pswf *ps, double lam, int nlev, orc_split3 *sp)
{
    memset(sp, 0, sizeof(*sp));
    sp->lam = lam;
    sp->nlev = nlev;
    sp->deg = ORC3_DEG;
    const int nc = ORC3_DEG + 1;
    sp->coef = (double *)calloc((size_t)nlev * nc, sizeof(double));
    sp->self = (double *)calloc((size_t)nlev, sizeof(double));
    double t[Y3_NGL * Y3_NPANEL], w[Y3_NGL * Y3_NPANEL];
    double f[ORC3_DEG + 1];
    for (int l = 0; l < nlev; ++l) {
        const int nq = y3_nodes(ps, lam * side(l), t, w);
        /* m_mu at the first-kind Chebyshev points of u = 2x^2 - 1 */
        for (int j = 0; j < nc; ++j) {
            const double u = cos(M_PI * (j + 0.5) / nc), x = sqrt(0.5 * (u + 1.0));
            double s = 0.0;
            for (int k = 0; k < nq; ++k) s += w[k] * sinc_t(t[k], x);
            f[j] = s;
        }
        for (int kk = 0; kk < nc; ++kk) {
            double s = 0.0;
            for (int j = 0; j < nc; ++j) s += f[j] * cos(M_PI * kk * (j + 0.5) / nc);
            sp->coef[(size_t)l * nc + kk] = (kk == 0 ? 1.0 : 2.0) * s / nc;
        }
        double s0 = 0.0;
        for (int k = 0; k < nq; ++k) s0 += w[k] * t[k];
        sp->self[l] = s0 / side(l); /* M_l(0) */
    }
    return 0;
}

void orc_y3_split_free(orc_split3 *sp)
{
    free(sp->coef);
    free(sp->self);
    memset(sp, 0, sizeof(*sp));
}

/* m_mu(x) of level l from the Chebyshev table (Clenshaw in u = 2x^2 - 1) */
double orc_y3_smooth(const orc_split3 *sp, int l, double x)
{
    const int nc = sp->deg + 1;
    const double *a = sp->coef + (size_t)l * nc;
    const double u = 2.0 * x * x - 1.0;
    double b1 = 0.0, b2 = 0.0;
    for (int k = nc - 1; k >= 1; --k) {
        const double b0 = a[k] + 2.0 * u * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return a[0] + u * b1 - b2;
}

double orc_y3_residual(const orc_split3 *sp, int l, double r)
{
    const double s = side(l), x = r / s;
    if (x >= 1.0) return 0.0;
    return exp(-sp->lam * r) / r - orc_y3_smooth(sp, l, x) / s;
}

/* plane-wave (trapezoidal) sums at a 3-D offset, for the pins */
double orc_y3_d_pw(const orc_pswf *ps, const orc_params *pr, double lam, int l, const double x[3])
{
    const double h = 2.0 * M_PI / (3.0 * side(l)), fac = pow(h / (2.0 * M_PI), 3);
    double s = 0.0;
    for (int m1 = -pr->nf; m1 <= pr->nf; ++m1)
        for (int m2 = -pr->nf; m2 <= pr->nf; ++m2)
            for (int m3 = -pr->nf; m3 <= pr->nf; ++m3) {
                const double k = h * sqrt((double)(m1 * m1 + m2 * m2 + m3 * m3));
                s += fac * orc_y3_dhat(ps, lam, l, k) * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
            }
    return s;
}

double orc_y3_w0_pw(const orc_pswf *ps, const orc_params *pr, double lam, const double x[3])
{
    const double h = pr->hw, fac = pow(h / (2.0 * M_PI), 3);
    double s = 0.0;
    for (int m1 = -pr->nw; m1 <= pr->nw; ++m1)
        for (int m2 = -pr->nw; m2 <= pr->nw; ++m2)
            for (int m3 = -pr->nw; m3 <= pr->nw; ++m3) {
                const double k = h * sqrt((double)(m1 * m1 + m2 * m2 + m3 * m3));
                s += fac * orc_y3_w0hat(ps, lam, k) * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
            }
    return s;
}

/* u_i = sum_{j != i, r_ij > 0} q_j e^{-lambda r_ij}/(4 pi r_ij), lambda in
 * input units, Neumaier sum */
void orc_direct_yuk3(double lam, int64_t n, const double *pts, const double *q, int64_t nt, const int64_t *tidx,
                     double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t tt = 0; tt < nt; ++tt) {
        const int64_t i = tidx[tt];
        double s = 0.0, comp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pts[3 * i] - pts[3 * j], dy = pts[3 * i + 1] - pts[3 * j + 1],
                         dz = pts[3 * i + 2] - pts[3 * j + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            const double v = q[j] * exp(-lam * r) / r, tsum = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - tsum) + v;
            else comp += (v - tsum) + s;
            s = tsum;
        }
        out[tt] = (s + comp) / (4.0 * M_PI);
    }
}
