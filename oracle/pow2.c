/*
 * pow2.c -- the 3-D kernel K(r) = 1/r^2 split in physical space with the
 * PSWF power-function window of Sec. 4.5 (eqs. powerfunctionpswfsplitting,
 * powerfunctionkernels, powerphil with alpha = 2):
 *   Phi(x) = (1/C_1) int_0^x t psi(t) dt for 0 <= x <= 1, 1 beyond,
 *            C_1 = int_0^1 t psi(t) dt;
 *   M_0(r) = Phi(r/s_0)/r^2,  D_l(r) = (Phi(r/s_{l+1}) - Phi(r/s_l))/r^2,
 *   R_L(r) = (1 - Phi(r/s_L))/r^2,  M_L(0) = psi(0)/(2 C_1 s_L^2).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * D_l(r) = 4^l D_0(2^l r), so Dhat_l(k) = 2^-l Dhat_0(2^-l k) and the
 * plane-wave weights (h_l/2pi)^3 Dhat_l(h_l |m|) are 4^l times level 0's.
 * Dhat_0(k) = (4 pi/k) int_0^1 D_0(r) r sin(kr) dr by Gauss-Legendre panels
 * (the paper gives no closed form for alpha = 2).
 *
 * The root: M_0 = 1/r^2 beyond s_0, so it is windowed in physical space,
 * W_0(r) = M_0(r) chi(r), with chi = 1 up to sqrt 3 (every offset inside the
 * unit box) and a smooth step to 0 over [sqrt 3, sqrt 3 + 2] built from the
 * 1/r split's window Phi_1 (the normalised integral of psi):
 *   chi(r) = (1 - sign(y) Phi_1(|y|))/2,  y = (r - sqrt 3) - 1.
 * (The mollified kernel of this split is not a convolution of 1/r^2 with a
 * compactly supported function, so the truncated-kernel construction of
 * Sec. 4.7 does not apply.)  W_0 vanishes beyond A = 2 + sqrt 3, so the
 * spacing h_W = 2 pi/(1 + A) = 2 pi/(3 + sqrt 3) keeps periodic images away
 * from offsets in the unit box, as for 1/r.  What_0 by radial quadrature.
 * Lengths in root-box units; the unit change is u = u'/S^2.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define P2_NGL 40   /* Gauss-Legendre nodes of the Phi integral (t psi(t) has degree < 80) */
#define P2_QGL 24   /* nodes per panel of the radial transforms */

static double side(int l) { return ldexp(1.0, -l); }

double orc_p2_c1(const orc_pswf *ps)
{
    double gx[P2_NGL], gw[P2_NGL];
    orc_gauss_legendre(P2_NGL, gx, gw);
    double s = 0.0;
    for (int i = 0; i < P2_NGL; ++i) {
        const double t = 0.5 * (gx[i] + 1.0);
        s += 0.5 * gw[i] * t * orc_pswf_eval(ps, t);
    }
    return s;
}

/* Phi by its defining integral (Gauss-Legendre on [0, x]) */
double orc_p2_phi_quad(const orc_pswf *ps, double x)
{
    if (x >= 1.0) return 1.0;
    if (x <= 0.0) return 0.0;
    double gx[P2_NGL], gw[P2_NGL];
    orc_gauss_legendre(P2_NGL, gx, gw);
    double s = 0.0;
    for (int i = 0; i < P2_NGL; ++i) {
        const double t = 0.5 * x * (gx[i] + 1.0);
        s += 0.5 * x * gw[i] * t * orc_pswf_eval(ps, t);
    }
    return s / orc_p2_c1(ps);
}

/* Phi(x)/x^2 is even and smooth: tabulated as a Chebyshev series in
 * u = 2x^2 - 1 from the defining integral at 48 nodes */
int orc_p2_init(const orc_pswf *ps, orc_pow2 *tb)
{
    memset(tb, 0, sizeof(*tb));
    tb->ps = ps;
    tb->c1 = orc_p2_c1(ps);
    const int nc = ORC_P2_NC;
    double f[ORC_P2_NC];
    for (int j = 0; j < nc; ++j) {
        const double u = cos(M_PI * (j + 0.5) / nc), x = sqrt(0.5 * (u + 1.0));
        f[j] = orc_p2_phi_quad(ps, x) / (x * x);
    }
    for (int k = 0; k < nc; ++k) {
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += f[j] * cos(M_PI * k * (j + 0.5) / nc);
        tb->coef[k] = (k == 0 ? 1.0 : 2.0) * s / nc;
    }
    return 0;
}

/* Phi(x)/x^2 on [0, 1] (Clenshaw) */
static double p2_g(const orc_pow2 *tb, double x)
{
    const double u = 2.0 * x * x - 1.0;
    double b1 = 0.0, b2 = 0.0;
    for (int k = ORC_P2_NC - 1; k >= 1; --k) {
        const double b0 = tb->coef[k] + 2.0 * u * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return tb->coef[0] + u * b1 - b2;
}

double orc_p2_phi(const orc_pow2 *tb, double x)
{
    if (x >= 1.0) return 1.0;
    if (x <= 0.0) return 0.0;
    return x * x * p2_g(tb, x);
}

double orc_p2_m0(const orc_pow2 *tb, int L) /* M_L(0) = psi(0)/(2 C_1 s_L^2) */
{
    const double s = side(L);
    return tb->ps->psi0 / (2.0 * tb->c1 * s * s);
}

double orc_p2_d(const orc_pow2 *tb, int l, double r)
{
    const double s0 = side(l), s1 = side(l + 1);
    if (r == 0.0) return orc_p2_m0(tb, l + 1) - orc_p2_m0(tb, l);
    return (orc_p2_phi(tb, r / s1) - orc_p2_phi(tb, r / s0)) / (r * r);
}

double orc_p2_r(const orc_pow2 *tb, int L, double r)
{
    const double x = r / side(L);
    if (x >= 1.0) return 0.0;
    return (1.0 - orc_p2_phi(tb, x)) / (r * r);
}

double orc_p2_w0(const orc_pow2 *tb, double r) /* M_0(r) chi(r) */
{
    const double a = sqrt(3.0);
    double chi = 1.0;
    if (r >= a + 2.0) return 0.0;
    if (r > a) {
        const double y = (r - a) - 1.0;
        chi = 0.5 * (1.0 - (y >= 0.0 ? 1.0 : -1.0) * orc_pswf_phi(tb->ps, fabs(y)));
    }
    const double m0 = (r == 0.0) ? orc_p2_m0(tb, 0) : orc_p2_phi(tb, r) / (r * r);
    return m0 * chi;
}

/* (4 pi/k) int_a^b f(r) r sin(kr) dr (k > 0), or 4 pi int f r^2 (k = 0), on
 * npan Gauss-Legendre panels */
static double radial_ft(double (*f)(const orc_pow2 *, double), const orc_pow2 *tb, double a, double b, int npan,
                        double k)
{
    double gx[P2_QGL], gw[P2_QGL];
    orc_gauss_legendre(P2_QGL, gx, gw);
    double s = 0.0;
    for (int pnl = 0; pnl < npan; ++pnl) {
        const double lo = a + (b - a) * pnl / npan, hi = a + (b - a) * (pnl + 1) / npan;
        for (int i = 0; i < P2_QGL; ++i) {
            const double r = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[i];
            const double w = 0.5 * (hi - lo) * gw[i];
            s += w * f(tb, r) * r * (k == 0.0 ? r : sin(k * r) / k);
        }
    }
    return 4.0 * M_PI * s;
}

static double d0_fn(const orc_pow2 *tb, double r) { return orc_p2_d(tb, 0, r); }

double orc_p2_dhat(const orc_pow2 *tb, int l, double k)
{
    /* D_0 is smooth on [0, 1/2] and on [1/2, 1] */
    const double k0 = k * side(l);
    const double v = radial_ft(d0_fn, tb, 0.0, 0.5, 12, k0) + radial_ft(d0_fn, tb, 0.5, 1.0, 12, k0);
    return side(l) * v;
}

double orc_p2_w0hat(const orc_pow2 *tb, double k)
{
    const double a = sqrt(3.0);
    return radial_ft(orc_p2_w0, tb, 0.0, 1.0, 16, k) + radial_ft(orc_p2_w0, tb, 1.0, a, 8, k) +
           radial_ft(orc_p2_w0, tb, a, a + 2.0, 16, k);
}

double orc_p2_d_pw(const orc_pow2 *tb, const orc_params *pr, int l, const double x[3])
{
    const double h = 2.0 * M_PI / (3.0 * side(l)), fac = pow(h / (2.0 * M_PI), 3);
    const int nf = pr->nf, maxk2 = 3 * nf * nf;
    double *memo = (double *)malloc((size_t)(maxk2 + 1) * sizeof(double));
    for (int k2 = 0; k2 <= maxk2; ++k2) memo[k2] = fac * orc_p2_dhat(tb, l, h * sqrt((double)k2));
    double s = 0.0;
    for (int m1 = -nf; m1 <= nf; ++m1)
        for (int m2 = -nf; m2 <= nf; ++m2)
            for (int m3 = -nf; m3 <= nf; ++m3)
                s += memo[m1 * m1 + m2 * m2 + m3 * m3] * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
    free(memo);
    return s;
}

double orc_p2_w0_pw(const orc_pow2 *tb, const orc_params *pr, const double x[3])
{
    const double h = pr->hw, fac = pow(h / (2.0 * M_PI), 3);
    const int nw = pr->nw, maxk2 = 3 * nw * nw;
    double *memo = (double *)malloc((size_t)(maxk2 + 1) * sizeof(double));
    for (int k2 = 0; k2 <= maxk2; ++k2) memo[k2] = fac * orc_p2_w0hat(tb, h * sqrt((double)k2));
    double s = 0.0;
    for (int m1 = -nw; m1 <= nw; ++m1)
        for (int m2 = -nw; m2 <= nw; ++m2)
            for (int m3 = -nw; m3 <= nw; ++m3)
                s += memo[m1 * m1 + m2 * m2 + m3 * m3] * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
    free(memo);
    return s;
}

/* u_i = sum_{j != i, r_ij > 0} q_j / r_ij^2, Neumaier sum */
void orc_direct_pow2(int64_t n, const double *pts, const double *q, int64_t nt, const int64_t *tidx, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t tt = 0; tt < nt; ++tt) {
        const int64_t i = tidx[tt];
        double s = 0.0, comp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pts[3 * i] - pts[3 * j], dy = pts[3 * i + 1] - pts[3 * j + 1],
                         dz = pts[3 * i + 2] - pts[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            const double v = q[j] / r2, tsum = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - tsum) + v;
            else comp += (v - tsum) + s;
            s = tsum;
        }
        out[tt] = s + comp;
    }
}
