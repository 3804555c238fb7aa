/*
 * split2.c -- 2-D kernels and their PSWF split in Fourier space.
 * TEST INFRASTRUCTURE ONLY (see oracle.h); FP64, plain loops.
 *
 * Kernels (input units): K(r) = -log(r)/(2 pi) (2-D Laplace) and
 * K(r) = K_0(lambda r) (2-D Yukawa).  Their transforms are 1/k^2 and
 * 2 pi/(k^2 + lambda^2); with kappa = sqrt(k^2 + lambda^2) the split of Sec.
 * 4.4 ("Kernel splitting using Gaussians or PSWFs in Fourier space", eq.
 * yukawaPSWFkernels) multiplies the transform by the mollifier
 * psi(kappa s_l/c)/psi(0), s_l = 2^{-l} being the box side at level l:
 *   Dhat_l(k) = a [psi(kappa s_{l+1}/c) - psi(kappa s_l/c)] / (psi(0) kappa^2),
 *   a = 1 (log) or 2 pi (K_0).
 * The root carries the windowed kernel of Sec. 4.7 ("Handling singularities
 * in Fourier space"): What_0 = psi(kappa s_0/c)/psi(0) * That(k), That being
 * the transform of K truncated at radius A = (1 + sqrt 2) s_0 (the Vico
 * truncation); for the log kernel
 *   That(k) = (1 - J_0(kA))/k^2 - A log(A) J_1(kA)/k,
 * and for K_0(lambda r)
 *   That(k) = 2 pi {1 + A [k J_1(kA) K_0(lambda A) - lambda J_0(kA) K_1(lambda A)]} / (k^2 + lambda^2).
 * The mollified kernel M_l = K - R_l is obtained from its transform by the
 * 2-D radial inverse transform f(r) = (1/2 pi) int_0^inf fhat(k) J_0(kr) k dk.
 * With x = r/s_l and t = k s_l:
 *   log:  R_l(r) = -log(x)/(2 pi) - m(x),
 *         m(x) = (1/2 pi) int_0^T psi(t/c)/psi(0) (J_0(tx) - J_0(t)) dt/t,
 *         (R_l vanishes at x = 1; m(x) = -log(x)/(2 pi) for x >= 1 to within
 *         the split's precision), M_l(0) = -log(s_l)/(2 pi) + m(0);
 *   K_0:  M_l(r) = int_0^T psi(sqrt(t^2 + mu^2)/c)/psi(0) J_0(tx) t/(t^2 + mu^2) dt,
 *         mu = lambda s_l, R_l(r) = K_0(lambda r) - M_l(r).
 * T is where the mollifier argument reaches 2 (|psi(2)/psi(0)| is below
 * 1e-9 at the Table 1 values of c); R_l is taken as 0 for r >= s_l.
 * The smooth parts m and M_l are even and entire in x; they are tabulated
 * once per level as Chebyshev series in u = 2 x^2 - 1 from values computed by
 * composite Gauss-Legendre quadrature on geometrically graded panels.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------- Bessel K_0, K_1
 * Small x: the ascending series K_0(x) = -(log(x/2) + gamma) I_0(x)
 * + sum_k (x^2/4)^k/(k!)^2 H_k and K_1(x) = (1/x) + I_1(x) log(x/2)
 * - (x/4) sum_k (x^2/4)^k/(k!(k+1)!) (psi(k+1) + psi(k+2)) (Abramowitz &
 * Stegun 9.6.13, 9.6.11).  Large x: the integral K_nu(x) = int_0^inf
 * exp(-x cosh t) cosh(nu t) dt by the trapezoidal rule, which converges
 * geometrically for this analytic, doubly exponentially decaying integrand. */
static const double EULER_GAMMA = 0.57721566490153286061;

static double k_integral(int nu, double x)
{
    const double h = 0.05;
    double s = 0.5 * exp(-x);
    for (int j = 1;; ++j) {
        double t = j * h, ch = cosh(t);
        double v = exp(-x * ch) * (nu ? cosh(t) : 1.0);
        s += v;
        if (x * ch > 745.0 || (v < 1e-300 && j > 10)) break;
    }
    return h * s;
}

double orc_bessel_k0(double x)
{
    if (x > 2.0) return k_integral(0, x);
    double y = 0.25 * x * x, term = 1.0, i0 = 1.0, sum = 0.0, H = 0.0;
    for (int k = 1; k < 60; ++k) {
        term *= y / ((double)k * k);
        H += 1.0 / k;
        i0 += term;
        sum += term * H;
        if (term < 1e-18 * i0) break;
    }
    return -(log(0.5 * x) + EULER_GAMMA) * i0 + sum;
}

double orc_bessel_k1(double x)
{
    if (x > 2.0) return k_integral(1, x);
    double y = 0.25 * x * x;
    /* I_1(x) = (x/2) sum_k y^k/(k!(k+1)!) */
    double term = 1.0, i1 = 1.0, s2 = 0.0;
    /* digamma(k+1) + digamma(k+2) with digamma(n) = -gamma + H_{n-1} */
    double Hk = 0.0;  /* H_k */
    s2 = (-EULER_GAMMA + Hk) + (-EULER_GAMMA + Hk + 1.0);
    double acc = s2;
    for (int k = 1; k < 60; ++k) {
        term *= y / ((double)k * (k + 1));
        Hk += 1.0 / k;
        i1 += term;
        acc += term * ((-EULER_GAMMA + Hk) + (-EULER_GAMMA + Hk + 1.0 / (k + 1)));
        if (term < 1e-18) break;
    }
    i1 *= 0.5 * x;
    return 1.0 / x + i1 * log(0.5 * x) - 0.25 * x * acc;
}

double orc2_kernel(int kern, double lam, double r)
{
    if (kern == ORC_LOG2) return -log(r) / (2.0 * M_PI);
    return orc_bessel_k0(lam * r);
}

/* Table 1 (c, nf, p) as in 3-D; the root window's spacing follows from its
 * support: W_0 vanishes beyond A + s_0 and offsets inside the unit box reach
 * 1 per axis, so the period 2 pi/h_W must be >= 1 + A + s_0 = 3 + sqrt 2. */
int orc_params2_for(double tol, orc_params *out)
{
    if (orc_params_for(tol, out)) return -1;
    out->hw = 2.0 * M_PI / (3.0 + sqrt(2.0));
    out->nw = (int)ceil(out->c / out->hw);
    return 0;
}

static double side(int l) { return ldexp(1.0, -l); }

double orc2_dhat(const orc_pswf *ps, int kern, double lam, int l, double k)
{
    const double a = (kern == ORC_LOG2) ? 1.0 : 2.0 * M_PI;
    const double lm = (kern == ORC_LOG2) ? 0.0 : lam;
    const double s0 = side(l), s1 = side(l + 1);
    const double kap2 = k * k + lm * lm;
    if (kap2 == 0.0) /* psi(x) = psi(0)(1 - (c2/c0) c^2 x^2/2 + ...) */
        return a * 0.5 * ps->c2 / ps->c0 * (s0 * s0 - s1 * s1);
    const double kap = sqrt(kap2);
    return a * (orc_pswf_eval_ext(ps, kap * s1 / ps->c) - orc_pswf_eval_ext(ps, kap * s0 / ps->c)) /
           (ps->psi0 * kap2);
}

static double bessel_j0(double x) { return j0(x); }
static double bessel_j1(double x) { return j1(x); }

double orc2_w0hat(const orc_pswf *ps, int kern, double lam, double k)
{
    const double A = 1.0 + sqrt(2.0); /* (1 + sqrt d) s_0 */
    double That;
    if (kern == ORC_LOG2) {
        if (k == 0.0) That = 0.25 * A * A - 0.5 * A * A * log(A);
        else That = (1.0 - bessel_j0(k * A)) / (k * k) - A * log(A) * bessel_j1(k * A) / k;
        return orc_pswf_eval_ext(ps, k * side(0) / ps->c) / ps->psi0 * That;
    }
    That = 2.0 * M_PI *
           (1.0 + A * (k * bessel_j1(k * A) * orc_bessel_k0(lam * A) - lam * bessel_j0(k * A) * orc_bessel_k1(lam * A))) /
           (k * k + lam * lam);
    return orc_pswf_eval_ext(ps, sqrt(k * k + lam * lam) * side(0) / ps->c) / ps->psi0 * That;
}

/* ---------------------------------------------- smooth parts by quadrature */
#define Q2_NGL 24
#define Q2_NPANEL 44

/* quadrature nodes on [0, T]: [0, T 2^-(NPANEL-1)], then panels doubling in length */
static void q2_nodes(double T, double *t, double *w)
{
    double gx[Q2_NGL], gw[Q2_NGL];
    orc_gauss_legendre(Q2_NGL, gx, gw);
    int k = 0;
    for (int pnl = 0; pnl < Q2_NPANEL; ++pnl) {
        double a = (pnl == 0) ? 0.0 : T * ldexp(1.0, pnl - Q2_NPANEL);
        double b = T * ldexp(1.0, pnl + 1 - Q2_NPANEL);
        for (int q = 0; q < Q2_NGL; ++q, ++k) {
            t[k] = 0.5 * (a + b) + 0.5 * (b - a) * gx[q];
            w[k] = 0.5 * (b - a) * gw[q];
        }
    }
}

/* the weight function of the smooth part, at the quadrature nodes */
static int q2_weights(const orc_pswf *ps, int kern, double mu, double *t, double *w)
{
    const double c = ps->c;
    double T;
    if (kern == ORC_LOG2) T = 2.0 * c;
    else {
        double T2 = 4.0 * c * c - mu * mu;
        if (T2 <= 0.0) return 0;
        T = sqrt(T2);
    }
    q2_nodes(T, t, w);
    const int nq = Q2_NGL * Q2_NPANEL;
    for (int k = 0; k < nq; ++k) {
        if (kern == ORC_LOG2) w[k] *= orc_pswf_eval_ext(ps, t[k] / c) / ps->psi0 / t[k] / (2.0 * M_PI);
        else {
            double kap2 = t[k] * t[k] + mu * mu;
            w[k] *= orc_pswf_eval_ext(ps, sqrt(kap2) / c) / ps->psi0 * t[k] / kap2;
        }
    }
    return nq;
}

double orc2_smooth_quad(const orc_pswf *ps, int kern, double mu, double x)
{
    double t[Q2_NGL * Q2_NPANEL], w[Q2_NGL * Q2_NPANEL];
    int nq = q2_weights(ps, kern, mu, t, w);
    double s = 0.0;
    for (int k = 0; k < nq; ++k) {
        if (kern == ORC_LOG2) s += w[k] * (bessel_j0(t[k] * x) - bessel_j0(t[k]));
        else s += w[k] * bessel_j0(t[k] * x);
    }
    return s;
}

int orc2_split_init(const orc_pswf *ps, int kern, double lam, int nlev, orc_split2 *sp)
{
    memset(sp, 0, sizeof(*sp));
    sp->kern = kern;
    sp->lam = lam;
    sp->nlev = nlev;
    sp->deg = ORC2_DEG;
    const int nc = ORC2_DEG + 1;
    sp->coef = (double *)calloc((size_t)nlev * nc, sizeof(double));
    sp->self = (double *)calloc((size_t)nlev, sizeof(double));
    double t[Q2_NGL * Q2_NPANEL], w[Q2_NGL * Q2_NPANEL];
    double f[ORC2_DEG + 1];
    for (int l = 0; l < nlev; ++l) {
        if (kern == ORC_LOG2 && l > 0) {
            memcpy(sp->coef + (size_t)l * nc, sp->coef, nc * sizeof(double));
            sp->self[l] = sp->self[0] - log(side(l)) / (2.0 * M_PI);
            continue;
        }
        const double mu = lam * side(l);
        int nq = q2_weights(ps, kern, mu, t, w);
        /* values at the Chebyshev points u_j of the first kind, x^2 = (u_j + 1)/2 */
        for (int j = 0; j < nc; ++j) {
            double u = cos(M_PI * (j + 0.5) / nc), x = sqrt(0.5 * (u + 1.0));
            double s = 0.0;
            for (int k = 0; k < nq; ++k) {
                if (kern == ORC_LOG2) s += w[k] * (bessel_j0(t[k] * x) - bessel_j0(t[k]));
                else s += w[k] * bessel_j0(t[k] * x);
            }
            f[j] = s;
        }
        /* a_k = (2/n) sum_j f_j T_k(u_j), a_0 halved */
        for (int kk = 0; kk < nc; ++kk) {
            double s = 0.0;
            for (int j = 0; j < nc; ++j) s += f[j] * cos(M_PI * kk * (j + 0.5) / nc);
            sp->coef[(size_t)l * nc + kk] = (kk == 0 ? 1.0 : 2.0) * s / nc;
        }
        /* value at x = 0 by the same quadrature */
        double s0 = 0.0;
        for (int k = 0; k < nq; ++k) {
            if (kern == ORC_LOG2) s0 += w[k] * (1.0 - bessel_j0(t[k]));
            else s0 += w[k];
        }
        sp->self[l] = (kern == ORC_LOG2) ? s0 - log(side(l)) / (2.0 * M_PI) : s0;
    }
    return 0;
}

void orc2_split_free(orc_split2 *sp)
{
    free(sp->coef);
    free(sp->self);
    memset(sp, 0, sizeof(*sp));
}

/* Chebyshev series of the smooth part at x = r/s_l (Clenshaw in u = 2x^2 - 1) */
double orc2_smooth(const orc_split2 *sp, int l, double x)
{
    const int nc = sp->deg + 1;
    const double *a = sp->coef + (size_t)l * nc;
    double u = 2.0 * x * x - 1.0, b1 = 0.0, b2 = 0.0;
    for (int k = nc - 1; k >= 1; --k) {
        double b0 = a[k] + 2.0 * u * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return a[0] + u * b1 - b2;
}

double orc2_residual(const orc_split2 *sp, int l, double r)
{
    const double s = side(l), x = r / s;
    if (x >= 1.0) return 0.0;
    if (sp->kern == ORC_LOG2) return -log(x) / (2.0 * M_PI) - orc2_smooth(sp, l, x);
    return orc_bessel_k0(sp->lam * r) - orc2_smooth(sp, l, x);
}

/* plane-wave sums (trapezoidal rule in k) at a 2-D offset, for the pins */
double orc2_d_pw(const orc_pswf *ps, const orc_params *pr, int kern, double lam, int l, const double x[2])
{
    const double h = 2.0 * M_PI / (3.0 * side(l)), fac = pow(h / (2.0 * M_PI), 2);
    double s = 0.0;
    for (int m1 = -pr->nf; m1 <= pr->nf; ++m1)
        for (int m2 = -pr->nf; m2 <= pr->nf; ++m2) {
            double k = h * sqrt((double)(m1 * m1 + m2 * m2));
            s += fac * orc2_dhat(ps, kern, lam, l, k) * cos(h * (m1 * x[0] + m2 * x[1]));
        }
    return s;
}

double orc2_w0_pw(const orc_pswf *ps, const orc_params *pr, int kern, double lam, const double x[2])
{
    const double h = pr->hw, fac = pow(h / (2.0 * M_PI), 2);
    double s = 0.0;
    for (int m1 = -pr->nw; m1 <= pr->nw; ++m1)
        for (int m2 = -pr->nw; m2 <= pr->nw; ++m2) {
            double k = h * sqrt((double)(m1 * m1 + m2 * m2));
            s += fac * orc2_w0hat(ps, kern, lam, k) * cos(h * (m1 * x[0] + m2 * x[1]));
        }
    return s;
}
