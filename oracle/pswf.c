/*
 * pswf.c -- PSWF psi_0^c, the PSWF kernel split of 1/r and its plane-wave
 * weights.  TEST INFRASTRUCTURE ONLY (see oracle.h); FP64, plain loops.
 *
 * psi_0^c is the first eigenfunction of F_c[phi](x) = int_{-1}^1 phi(t)
 * e^{icxt} dt (Appendix, PSWFs of order zero).  It is computed as the ground
 * state of the prolate Sturm-Liouville operator that commutes with F_c,
 * expanded in normalised Legendre polynomials (the classical Bouwkamp /
 * Legendre-Galerkin method): the even-index matrix is symmetric tridiagonal;
 * its smallest eigenvalue is found by Sturm-sequence bisection and its
 * eigenvector by shifted inverse iteration.  Outside [-1,1] psi is defined by
 * the eigen-relation psi(x) = (1/lambda_0) int_{-1}^1 psi(t) cos(cxt) dt.
 *
 * Kernel split (Sec. 3.7, eq. newkernels), for box side s_l = 2^{-l}:
 *   Phi(x) = (1/c_0) int_0^{min(x,1)} psi,
 *   W_0(r) = Phi(r/s_0)/r,  D_l(r) = (Phi(r/s_{l+1}) - Phi(r/s_l))/r,
 *   R_L(r) = (1 - Phi(r/s_L))/r.
 * Fourier transforms: eq. differencekernelft3 for D_l; the windowed W_0 is the
 * mollifier transform psi(k s_0/c)/psi(0) times the transform of 1/r
 * truncated at A = (1 + sqrt 3) s_0 (Sec. 4.7, "Handling singularities in
 * Fourier space", and the Vico truncation remark of Sec. 3.1), which is
 * 8 pi sin^2(kA/2)/k^2.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Gauss-Legendre nodes and weights on [-1,1] by Newton's method on P_n. */
void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Matrix of the prolate operator  -d/dx((1-x^2) d/dx) + c^2 x^2  in the
 * basis sqrt(k+1/2) P_k, restricted to even k = 2i. */
static void prolate_tridiag(double c, int K, double *d, double *e)
{
    for (int i = 0; i < K; ++i) {
        double k = 2.0 * i;
        d[i] = k * (k + 1.0) + c * c * (2.0 * k * (k + 1.0) - 1.0) /
                                   ((2.0 * k + 3.0) * (2.0 * k - 1.0));
        e[i] = c * c * (k + 1.0) * (k + 2.0) /
               ((2.0 * k + 3.0) * sqrt((2.0 * k + 1.0) * (2.0 * k + 5.0)));
    }
}

/* number of eigenvalues of the tridiagonal (d, e) strictly below x */
static int sturm_count(int K, const double *d, const double *e, double x)
{
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) cnt++;
    for (int i = 1; i < K; ++i) {
        double den = (q == 0.0) ? 1e-300 : q;
        q = d[i] - x - e[i - 1] * e[i - 1] / den;
        if (q < 0) cnt++;
    }
    return cnt;
}

/* Legendre P_0..P_kmax at x */
static void legendre_all(int kmax, double x, double *P)
{
    P[0] = 1.0;
    if (kmax >= 1) P[1] = x;
    for (int k = 2; k <= kmax; ++k)
        P[k] = ((2.0 * k - 1.0) * x * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
}

double orc_pswf_eval(const orc_pswf *ps, double x)
{
    int kmax = 2 * (ps->nterm - 1) + 1;
    double P[2 * ORC_PSWF_MAXTERM + 2];
    legendre_all(kmax, x, P);
    double s = 0.0;
    for (int i = 0; i < ps->nterm; ++i) {
        int k = 2 * i;
        s += ps->coef[i] * sqrt(k + 0.5) * P[k];
    }
    return s;
}

int orc_pswf_init(double c, orc_pswf *ps)
{
    memset(ps, 0, sizeof(*ps));
    ps->c = c;
    const int K = ORC_PSWF_MAXTERM;
    double d[ORC_PSWF_MAXTERM], e[ORC_PSWF_MAXTERM];
    prolate_tridiag(c, K, d, e);

    /* Gershgorin interval, then bisection for the smallest eigenvalue. */
    double lo = d[0] - fabs(e[0]), hi = d[0] + fabs(e[0]);
    for (int i = 1; i < K; ++i) {
        double r = fabs(e[i - 1]) + (i < K - 1 ? fabs(e[i]) : 0.0);
        if (d[i] - r < lo) lo = d[i] - r;
        if (d[i] + r > hi) hi = d[i] + r;
    }
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (sturm_count(K, d, e, mid) >= 1) hi = mid; else lo = mid;
        if (hi - lo <= 1e-15 * fabs(hi)) break;
    }
    double chi = 0.5 * (lo + hi);
    ps->chi = chi;

    /* Shifted inverse iteration; (T - sigma I) is positive definite for a
     * shift just below the smallest eigenvalue, so an LDL^T sweep is stable. */
    double sigma = chi - 1e-9 * (1.0 + fabs(chi));
    double v[ORC_PSWF_MAXTERM], dd[ORC_PSWF_MAXTERM], l[ORC_PSWF_MAXTERM];
    for (int i = 0; i < K; ++i) v[i] = 1.0;
    dd[0] = d[0] - sigma;
    for (int i = 1; i < K; ++i) {
        l[i] = e[i - 1] / dd[i - 1];
        dd[i] = d[i] - sigma - l[i] * e[i - 1];
    }
    for (int it = 0; it < 4; ++it) {
        for (int i = 1; i < K; ++i) v[i] -= l[i] * v[i - 1];
        for (int i = 0; i < K; ++i) v[i] /= dd[i];
        for (int i = K - 2; i >= 0; --i) v[i] -= l[i + 1] * v[i + 1];
        double nrm = 0.0;
        for (int i = 0; i < K; ++i) nrm += v[i] * v[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < K; ++i) v[i] /= nrm;
    }
    /* keep the terms that matter in double precision */
    double vmax = 0.0;
    for (int i = 0; i < K; ++i) if (fabs(v[i]) > vmax) vmax = fabs(v[i]);
    int nterm = K;
    while (nterm > 1 && fabs(v[nterm - 1]) < 1e-20 * vmax) nterm--;
    ps->nterm = nterm;
    for (int i = 0; i < K; ++i) ps->coef[i] = (i < nterm) ? v[i] : 0.0;
    if (orc_pswf_eval(ps, 0.0) < 0)
        for (int i = 0; i < nterm; ++i) ps->coef[i] = -ps->coef[i];
    ps->psi0 = orc_pswf_eval(ps, 0.0);

    /* c_0 = int_0^1 psi, c_2 = int_0^1 x^2 psi (Gauss-Legendre on [0,1]) */
    {
        double gx[128], gw[128];
        orc_gauss_legendre(128, gx, gw);
        double s0 = 0.0, s2 = 0.0;
        for (int q = 0; q < 128; ++q) {
            double t = 0.5 * (gx[q] + 1.0);
            double f = orc_pswf_eval(ps, t);
            s0 += 0.5 * gw[q] * f;
            s2 += 0.5 * gw[q] * t * t * f;
        }
        ps->c0 = s0;
        ps->c2 = s2;
    }
    /* lambda_0 from the eigen-relation at x = 0: int_{-1}^1 psi = lambda_0 psi(0) */
    ps->lambda0 = 2.0 * ps->c0 / ps->psi0;

    orc_gauss_legendre(ORC_GL_EXT, ps->glx, ps->glw);
    for (int q = 0; q < ORC_GL_EXT; ++q)
        ps->glpsi[q] = orc_pswf_eval(ps, ps->glx[q]);
    return 0;
}

double orc_pswf_eval_ext(const orc_pswf *ps, double x)
{
    if (fabs(x) <= 1.0) return orc_pswf_eval(ps, x);
    double s = 0.0;
    for (int q = 0; q < ORC_GL_EXT; ++q)
        s += ps->glw[q] * ps->glpsi[q] * cos(ps->c * x * ps->glx[q]);
    return s / ps->lambda0;
}

/* Phi(x) = (1/c_0) int_0^{min(x,1)} psi, using the Legendre antiderivative
 * int_0^x P_k = (P_{k+1}(x) - P_{k-1}(x)) / (2k+1) for even k >= 2. */
double orc_pswf_phi(const orc_pswf *ps, double x)
{
    if (x >= 1.0) return 1.0;
    if (x <= 0.0) return 0.0;
    int kmax = 2 * (ps->nterm - 1) + 1;
    double P[2 * ORC_PSWF_MAXTERM + 2];
    legendre_all(kmax, x, P);
    double s = ps->coef[0] * sqrt(0.5) * x;
    for (int i = 1; i < ps->nterm; ++i) {
        int k = 2 * i;
        s += ps->coef[i] * sqrt(k + 0.5) * (P[k + 1] - P[k - 1]) / (2.0 * k + 1.0);
    }
    return s / ps->c0;
}

static double side(int l) { return ldexp(1.0, -l); }

double orc_split_w0(const orc_pswf *ps, double r)
{
    if (r == 0.0) return ps->psi0 / ps->c0;
    return orc_pswf_phi(ps, r / side(0)) / r;
}

double orc_split_d(const orc_pswf *ps, int l, double r)
{
    if (r == 0.0) return ps->psi0 / ps->c0 * (1.0 / side(l + 1) - 1.0 / side(l));
    return (orc_pswf_phi(ps, r / side(l + 1)) - orc_pswf_phi(ps, r / side(l))) / r;
}

double orc_split_r(const orc_pswf *ps, int L, double r)
{
    return (1.0 - orc_pswf_phi(ps, r / side(L))) / r;
}

double orc_split_m0(const orc_pswf *ps, int L)
{
    return ps->psi0 / (ps->c0 * side(L));
}

double orc_dhat(const orc_pswf *ps, int l, double k)
{
    double s0 = side(l), s1 = side(l + 1);
    if (k == 0.0) return 2.0 * M_PI * ps->c2 / ps->c0 * (s0 * s0 - s1 * s1);
    return 4.0 * M_PI / ps->psi0 *
           (orc_pswf_eval_ext(ps, k * s1 / ps->c) - orc_pswf_eval_ext(ps, k * s0 / ps->c)) /
           (k * k);
}

double orc_w0hat(const orc_pswf *ps, double k)
{
    double A = 1.0 + sqrt(3.0); /* (1 + sqrt d) s_0 */
    if (k == 0.0) return 2.0 * M_PI * A * A;
    double sn = sin(k * A / 2.0);
    return 8.0 * M_PI * sn * sn / (k * k) * orc_pswf_eval_ext(ps, k * side(0) / ps->c) / ps->psi0;
}

/* D_l(x) ~ sum_m (h_l/2pi)^3 Dhat_l(h_l |m|) e^{i h_l m.x},  h_l = 2pi/(3 s_l) */
double orc_split_d_pw(const orc_pswf *ps, const orc_params *pr, int l, const double x[3])
{
    double h = 2.0 * M_PI / (3.0 * side(l));
    double fac = pow(h / (2.0 * M_PI), 3);
    double s = 0.0;
    for (int m1 = -pr->nf; m1 <= pr->nf; ++m1)
        for (int m2 = -pr->nf; m2 <= pr->nf; ++m2)
            for (int m3 = -pr->nf; m3 <= pr->nf; ++m3) {
                double k = h * sqrt((double)(m1 * m1 + m2 * m2 + m3 * m3));
                s += fac * orc_dhat(ps, l, k) * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
            }
    return s;
}

double orc_split_w0_pw(const orc_pswf *ps, const orc_params *pr, const double x[3])
{
    double h = pr->hw;
    double fac = pow(h / (2.0 * M_PI), 3);
    double s = 0.0;
    for (int m1 = -pr->nw; m1 <= pr->nw; ++m1)
        for (int m2 = -pr->nw; m2 <= pr->nw; ++m2)
            for (int m3 = -pr->nw; m3 <= pr->nw; ++m3) {
                double k = h * sqrt((double)(m1 * m1 + m2 * m2 + m3 * m3));
                s += fac * orc_w0hat(ps, k) * cos(h * (m1 * x[0] + m2 * x[1] + m3 * x[2]));
            }
    return s;
}

/* Any (c, nf, p), e.g. a caller's choice for a tolerance off the table; the
 * root window's spacing follows from its support as for the table rows (in
 * d dimensions W_0 vanishes beyond A + s_0 = 2 + sqrt d and offsets inside
 * the unit box reach 1 per axis). */
int orc_params_set(double tol, double c, int nf, int p, int dim, orc_params *out)
{
    if (!(c > 0) || nf < 1 || p < 2 || (dim != 2 && dim != 3)) return -1;
    out->tol = tol;
    out->c = c;
    out->nf = nf;
    out->p = p;
    out->hw = 2.0 * M_PI / (3.0 + sqrt((double)dim));
    out->nw = (int)ceil(c / out->hw);
    return 0;
}

/* Table 1 of the paper (c, N_1 = 2 nf + 1, p) and one row of our own for the
 * mixed-precision tolerance 1e-5 (c = log(1/eps), the rule of eq.
 * pswfcvalue). */
int orc_params_for(double tol, orc_params *out)
{
    static const struct { double tol, c; int nf, p; } rows[] = {
        {1e-3, 7.2462000846862793, 6, 9},
        {1e-5, 11.512925464970229, 10, 15},
        {1e-6, 13.739999771118164, 12, 18},
        {1e-9, 20.736000061035156, 19, 28},
        {1e-12, 27.870000839233398, 26, 38},
    };
    for (unsigned i = 0; i < sizeof(rows) / sizeof(rows[0]); ++i) {
        if (fabs(log10(tol) - log10(rows[i].tol)) < 1e-3) {
            out->tol = tol;
            out->c = rows[i].c;
            out->nf = rows[i].nf;
            out->p = rows[i].p;
            /* W_0 is supported on r <= A + s_0 with A = (1 + sqrt 3) s_0 and
             * coordinate offsets within the unit box are <= 1, so the period
             * 2 pi / h must be >= 1 + A + s_0 = 3 + sqrt 3. */
            out->hw = 2.0 * M_PI / (3.0 + sqrt(3.0));
            out->nw = (int)ceil(out->c / out->hw);
            return 0;
        }
    }
    return -1;
}
