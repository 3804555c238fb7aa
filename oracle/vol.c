/*
 * vol.c -- plain FP64 oracle for the DMK volume potential ("box code")
 *
 *     u(x) = int_{B_0} rho(y) / (4 pi |x - y|) dy,   B_0 = [-1/2, 1/2]^3,
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): nothing in the product library
 * links or calls this file.
 *
 * What it follows:
 *   - The Gaussian multilevel split of 1/r (Sec. 3.2, eqs. mlks, kerneldef,
 *     deltavalue): W_0 ~ erf(r/sigma_0)/r, D_l = (erf(r/sigma_{l+1}) -
 *     erf(r/sigma_l))/r, R_L = erfc(r/sigma_L)/r, sigma_0 = 1/sqrt(log(1/eps)),
 *     sigma_l = sigma_0 / 2^l.  Fourier transforms: erf(r/s)/r has 3-D
 *     transform 4 pi exp(-k^2 s^2/4)/k^2; the root kernel is the truncated 1/r
 *     (radius A = sqrt(3) + 1) times that Gaussian factor, whose truncated-1/r
 *     transform is 8 pi sin^2(kA/2)/k^2 (Sec. 3.1, the windowed kernel).
 *   - Sec. 3.6 "Modification of DMK for continuous sources":
 *       * an adaptive level-restricted tree that resolves rho by tensor
 *         polynomials of degree q-1 on every leaf;
 *       * proxy charges of a leaf = scaled Gauss-Legendre weights times rho at
 *         the Legendre nodes, anterpolated to the Chebyshev proxy grid
 *         (subsection "Creating proxy charges");
 *       * local expansions evaluated on the leaf's tensor grid;
 *       * the residual kernel as a continuous sum of Gaussians (eq.
 *         localkernel), discretised by quadrature in t; every Gaussian is a
 *         product of 1-D factors, so a (source leaf, target leaf) pair costs
 *         three 1-D matrices per Gaussian (subsection "Approximation of the
 *         local interactions").
 *   - Sec. 4.4 "Sum-of-Gaussians approximation": Gaussians narrow enough
 *     (t >= t_a with (4/(t_a R)^2)^3 < eps) are integrated over R^3 through
 *     the expansion rho + Delta rho/(4 t^2) + Delta^2 rho/(32 t^4) of the
 *     Gaussian convolution.
 *
 *   - At tol 1e-6, the PSWF split of Sec. 3.7 instead (the remark closing
 *     Sec. 3.6 proposes it, with Gaussians for the residual only): D_l and
 *     the windowed W_0 of the point code (p = 18, n_f = 12); the residual
 *     R_L = (1 - Phi(r/s_L))/r, in x = r/s_L, is
 *       h(x) + (2/sqrt pi) int_{theta1}^{t_a s_L} e^{-x^2 t^2} dt + erfc(t_a r)/r,
 *     h(x) = (erf(theta1 x) - Phi(x))/x: the integral is the same log-t
 *     quadrature (10 nodes on panels of width <= 1.4), the last term the same asymptotic
 *     part, and h is a sum of nfit Gaussians fitted by least squares
 *     (Sec. 3.6 asks for a sum of Gaussians and leaves its construction
 *     open; see vfit below for the nodes and the sample grid).
 *
 * Readings where the paper leaves a choice open (each is also a choice of
 * the GPU path, made independently there):
 *   - leaf nodes: first-kind Chebyshev points cos(pi (i + 1/2)/q) per axis;
 *   - refinement: a box is split when the sum of |c_ijk| over its Chebyshev
 *     coefficients with max(i,j,k) >= q-2 exceeds tol * rho_scale, while its
 *     level is below min_level, or while it contains a caller-given feature
 *     point (x, y, z, h) with h below its side (lo <= x < hi per axis): node
 *     samples cannot see features much narrower than the node spacing; then
 *     the minimal 2:1 balanced refinement (face, edge and corner adjacency);
 *   - proxy charges use p Gauss-Legendre nodes per axis (exact for the
 *     degree (p-1) + (q-1) products);
 *   - residual pairs: the source-centric lists of the point code (targets in
 *     the colleagues' subtrees and in coarse-neighbour leaves), minus pairs of
 *     boxes whose distance is at least the source box side (there every
 *     Gaussian of R_L is below eps);
 *   - the t-integral of R_L runs from 1/sigma_{L(source)} to
 *     t_a = 2 eps^(-1/6) 2^{L(target)} on panels of width 1 in log t, 5
 *     Gauss-Legendre nodes each (the sum reproduces erfc(r/sigma)/r -
 *     erfc(t_a r)/r to 3e-6 of 1/r, far below eps = 1e-3); beyond t_a the
 *     expansion above (to the Delta^2 term) with the derivatives of the
 *     target leaf's polynomial.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cheb.h"
#include "oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

#define VKB 21 /* key bits per axis */

/* ------------------------------------------------------------- parameters */
/* Least squares min |A w - b| by Householder QR (A is m x n, row-major,
 * m >= n, overwritten); w gets the n unknowns. */
static int lsq_householder(int m, int n, double *A, double *b, double *w)
{
    for (int k = 0; k < n; ++k) {
        double nrm = 0.0;
        for (int i = k; i < m; ++i) nrm += A[i * n + k] * A[i * n + k];
        nrm = sqrt(nrm);
        if (nrm == 0.0) return -1;
        const double alpha = A[k * n + k] > 0 ? -nrm : nrm;
        /* v = a_k - alpha e_k, stored in column k below the diagonal */
        A[k * n + k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < m; ++i) vv += A[i * n + k] * A[i * n + k];
        for (int j = k + 1; j < n; ++j) {
            double d = 0.0;
            for (int i = k; i < m; ++i) d += A[i * n + k] * A[i * n + j];
            d *= 2.0 / vv;
            for (int i = k; i < m; ++i) A[i * n + j] -= d * A[i * n + k];
        }
        double d = 0.0;
        for (int i = k; i < m; ++i) d += A[i * n + k] * b[i];
        d *= 2.0 / vv;
        for (int i = k; i < m; ++i) b[i] -= d * A[i * n + k];
        A[k * n + k] = alpha; /* R's diagonal */
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * w[j];
        w[k] = s / A[k * n + k];
    }
    return 0;
}

/* Sec. 3.6 asks for a sum of Gaussians for the residual kernel on [eps_0, 1]
 * and leaves the construction open.  With the PSWF split (Sec. 3.7) the
 * residual of level L is R_L(r) = (1 - Phi(r/s_L))/r.  In x = r/s_L,
 *   (1 - Phi(x))/x = h(x) + (2/sqrt pi) int_{theta1}^{tau} e^{-x^2 t^2} dt
 *                  + erfc(tau x)/x,     h(x) = (erf(theta1 x) - Phi(x))/x,
 * tau = t_a s_L: the last term is the asymptotic part (Sec. 4.4), the
 * middle one the quadrature in log t, and h -- bounded, even, and zero to
 * erfc(theta1) beyond x = 1 -- is fitted by nfit Gaussians e^{-x^2 t_i^2}
 * with fixed t_i (geometric from 0.5 to 10) by least squares on 2200 equal
 * steps of [0, 5.5] (the largest node distance of a near pair is below
 * 3 sqrt 3 source sides). */
static double fit_target(const orc_pswf *ps, const orc_vparams *vp, double x)
{
    if (x == 0.0) return 2.0 * vp->theta1 / sqrt(M_PI) - ps->psi0 / ps->c0;
    return (erf(vp->theta1 * x) - orc_pswf_phi(ps, x)) / x;
}

double orc_vfit_target(const orc_vparams *vp, double x)
{
    orc_pswf ps;
    if (vp->split != 1 || orc_pswf_init(vp->c, &ps) != 0) return NAN;
    return fit_target(&ps, vp, x);
}

static int vfit(orc_vparams *vp)
{
    const int m = 2200, n = vp->nfit;
    orc_pswf ps;
    if (n < 2 || n > ORC_VFIT_MAX || orc_pswf_init(vp->c, &ps) != 0) return -1;
    double *A = (double *)malloc((size_t)m * n * sizeof(double));
    double *b = (double *)malloc((size_t)m * sizeof(double));
    double *x = (double *)malloc((size_t)m * sizeof(double));
    for (int i = 0; i < n; ++i) vp->fit_t[i] = 0.5 * pow(20.0, (double)i / (n - 1));
    for (int j = 0; j < m; ++j) {
        x[j] = 5.5 * j / (m - 1);
        b[j] = fit_target(&ps, vp, x[j]);
        for (int i = 0; i < n; ++i) A[j * n + i] = exp(-x[j] * x[j] * vp->fit_t[i] * vp->fit_t[i]);
    }
    int rc = lsq_householder(m, n, A, b, vp->fit_w);
    vp->fit_err = 0.0;
    for (int j = 0; j < m && rc == 0; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += vp->fit_w[i] * exp(-x[j] * x[j] * vp->fit_t[i] * vp->fit_t[i]);
        double e = fabs(s - fit_target(&ps, vp, x[j]));
        if (e > vp->fit_err) vp->fit_err = e;
    }
    free(A);
    free(b);
    free(x);
    return rc;
}

int orc_vparams_for(double tol, int q, orc_vparams *vp)
{
    memset(vp, 0, sizeof(*vp));
    if (!(tol == 1e-3 || tol == 1e-6)) return -1;
    if (q < 2 || q > 16) return -1;
    vp->tol = tol;
    vp->q = q;
    vp->sigma0 = 1.0 / sqrt(log(1.0 / tol));
    vp->p = 18;
    vp->nf = 12;
    vp->nleg = 18;
    vp->tau_a = 2.0 * pow(tol, -1.0 / 6.0);
    vp->tpan_gl = 5;
    if (tol == 1e-3) {
        vp->nw = 14;
        vp->hw = 2.0 * M_PI / (2.0 * sqrt(3.0) + 2.0);
        vp->tpan_w = 1.0;
        return 0;
    }
    orc_params pr;
    if (orc_params_for(1e-6, &pr) != 0 || pr.p != 18 || pr.nf != 12) return -1;
    vp->split = 1;
    vp->c = pr.c;
    vp->nw = pr.nw;
    vp->hw = pr.hw;
    vp->tpan_gl = 10; /* one panel of 10 nodes covers [theta1, t_a s_L] = [5, 20] */
    vp->tpan_w = 1.4;
    vp->theta1 = 5.0;
    vp->nfit = 20;
    return vfit(vp);
}

static double sig(const orc_vparams *vp, int l) { return ldexp(vp->sigma0, -l); }

/* ------------------------------------------------------ Gaussian split */
double orc_gsplit_m(const orc_vparams *vp, int l, double r)
{
    double s = sig(vp, l);
    if (r == 0.0) return 2.0 / (sqrt(M_PI) * s);
    return erf(r / s) / r;
}

double orc_gsplit_d(const orc_vparams *vp, int l, double r)
{
    double s0 = sig(vp, l), s1 = sig(vp, l + 1);
    if (r == 0.0) return 2.0 / sqrt(M_PI) * (1.0 / s1 - 1.0 / s0);
    return (erfc(r / s0) - erfc(r / s1)) / r;
}

double orc_gsplit_r(const orc_vparams *vp, int l, double r) { return erfc(r / sig(vp, l)) / r; }

double orc_gdhat(const orc_vparams *vp, int l, double k)
{
    double s0 = sig(vp, l), s1 = sig(vp, l + 1);
    if (k == 0.0) return M_PI * (s0 * s0 - s1 * s1);
    /* 4 pi (e^{-k^2 s1^2/4} - e^{-k^2 s0^2/4}) / k^2, without cancellation */
    double a = 0.25 * k * k * s1 * s1, b = 0.25 * k * k * (s0 * s0 - s1 * s1);
    return 4.0 * M_PI * exp(-a) * (-expm1(-b)) / (k * k);
}

double orc_gw0hat(const orc_vparams *vp, double k)
{
    const double A = sqrt(3.0) + 1.0;
    double g = exp(-0.25 * k * k * vp->sigma0 * vp->sigma0);
    if (k == 0.0) return 2.0 * M_PI * A * A;
    double sn = sin(0.5 * k * A);
    return 8.0 * M_PI * sn * sn / (k * k) * g;
}

double orc_gsplit_d_pw(const orc_vparams *vp, int l, const double x[3])
{
    const int nf = vp->nf;
    const double s = ldexp(1.0, -l), h = 2.0 * M_PI / (3.0 * s), fac = pow(h / (2.0 * M_PI), 3);
    double acc = 0.0;
    for (int a = -nf; a <= nf; ++a)
        for (int b = -nf; b <= nf; ++b)
            for (int c = -nf; c <= nf; ++c) {
                double k = h * sqrt((double)(a * a + b * b + c * c));
                acc += fac * orc_gdhat(vp, l, k) * cos(h * (a * x[0] + b * x[1] + c * x[2]));
            }
    return acc;
}

double orc_gsplit_w0_pw(const orc_vparams *vp, const double x[3])
{
    const int nw = vp->nw;
    const double h = vp->hw, fac = pow(h / (2.0 * M_PI), 3);
    double acc = 0.0;
    for (int a = -nw; a <= nw; ++a)
        for (int b = -nw; b <= nw; ++b)
            for (int c = -nw; c <= nw; ++c) {
                double k = h * sqrt((double)(a * a + b * b + c * c));
                acc += fac * orc_gw0hat(vp, k) * cos(h * (a * x[0] + b * x[1] + c * x[2]));
            }
    return acc;
}

/* Sum of Gaussians for (2/sqrt(pi)) int_{t_lo}^{t_hi} exp(-r^2 t^2) dt: Gauss-
 * Legendre in u = log t on equal panels of width <= tpan_w.  Returns the
 * number of nodes (t, w need room for it). */
int orc_vsog(const orc_vparams *vp, double t_lo, double t_hi, double *t, double *w)
{
    if (!(t_hi > t_lo)) return 0;
    const double u0 = log(t_lo), u1 = log(t_hi);
    int npan = (int)ceil((u1 - u0) / vp->tpan_w - 1e-12);
    if (npan < 1) npan = 1;
    const double hp = (u1 - u0) / npan;
    double gx[32], gw[32];
    orc_gauss_legendre(vp->tpan_gl, gx, gw);
    int n = 0;
    for (int k = 0; k < npan; ++k)
        for (int j = 0; j < vp->tpan_gl; ++j) {
            double u = u0 + hp * (k + 0.5 * (gx[j] + 1.0));
            t[n] = exp(u);
            w[n] = 2.0 / sqrt(M_PI) * t[n] * 0.5 * hp * gw[j];
            ++n;
        }
    return n;
}

int orc_vsog_count(const orc_vparams *vp, double t_lo, double t_hi)
{
    if (!(t_hi > t_lo)) return 0;
    int npan = (int)ceil((log(t_hi) - log(t_lo)) / vp->tpan_w - 1e-12);
    if (npan < 1) npan = 1;
    return npan * vp->tpan_gl;
}

/* int_{-1}^{1} exp(-(xi - eta)^2 tau^2) L_b(eta) d eta for all b, where L_b is
 * the Lagrange basis of the q Chebyshev nodes; 64-point Gauss-Legendre on the
 * part of [-1,1] within 7/tau of xi (the rest is below e^-49). */
void orc_vgauss_row(const cheb_t *chq, double xi, double tau, double *out)
{
    const int q = chq->p;
    for (int b = 0; b < q; ++b) out[b] = 0.0;
    double lo = xi - 7.0 / tau, hi = xi + 7.0 / tau;
    if (lo < -1.0) lo = -1.0;
    if (hi > 1.0) hi = 1.0;
    if (!(hi > lo)) return;
    double gx[64], gw[64];
    orc_gauss_legendre(64, gx, gw);
    double L[64];
    for (int n = 0; n < 64; ++n) {
        double eta = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[n];
        double g = exp(-(xi - eta) * (xi - eta) * tau * tau) * 0.5 * (hi - lo) * gw[n];
        cheb_interp_row(chq, eta, L);
        for (int b = 0; b < q; ++b) out[b] += g * L[b];
    }
}

/* ------------------------------------------------------------------- tree */
static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < VKB; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

/* Morton key of cell (i,j,k) at level l, at VKB bits per axis (x most
 * significant within each bit triple) */
static uint64_t vkey(int l, const int32_t c[3])
{
    int sh = VKB - l;
    return (spread3((uint64_t)c[0] << sh) << 2) | (spread3((uint64_t)c[1] << sh) << 1) |
           spread3((uint64_t)c[2] << sh);
}

/* code unique to (level, cell): level in the top bits, level key below */
static uint64_t vcode(int l, const int32_t c[3]) { return ((uint64_t)l << 58) | (vkey(l, c) >> (3 * (VKB - l))); }

typedef struct { int32_t l, c[3]; } vbox;

static int u64cmp(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static int has_code(const uint64_t *s, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = (lo + hi) / 2;
        if (s[m] < v) lo = m + 1;
        else hi = m;
    }
    return lo < n && s[lo] == v;
}

static void node_coord(int q, int l, const int32_t c[3], int a, int b, int d, double out[3])
{
    const double s = ldexp(1.0, -l);
    int ab[3] = {a, b, d};
    for (int k = 0; k < 3; ++k) out[k] = -0.5 + (c[k] + 0.5) * s + 0.5 * s * cos(M_PI * (ab[k] + 0.5) / q);
}

/* sum of |c_ijk| with max(i,j,k) >= q-2 for the Chebyshev interpolant of f */
static double tail_coef(int q, const double *f)
{
    double Cm[16 * 16];
    for (int i = 0; i < q; ++i)
        for (int a = 0; a < q; ++a) Cm[i * q + a] = (i ? 2.0 : 1.0) / q * cos(i * M_PI * (a + 0.5) / q);
    int q3 = q * q * q;
    double *t1 = (double *)malloc((size_t)q3 * sizeof(double)), *t2 = (double *)malloc((size_t)q3 * sizeof(double));
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int k = 0; k < q; ++k) {
                double s = 0.0;
                for (int c = 0; c < q; ++c) s += Cm[k * q + c] * f[(a * q + b) * q + c];
                t1[(a * q + b) * q + k] = s;
            }
    for (int a = 0; a < q; ++a)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                double s = 0.0;
                for (int b = 0; b < q; ++b) s += Cm[j * q + b] * t1[(a * q + b) * q + k];
                t2[(a * q + j) * q + k] = s;
            }
    double eta = 0.0;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                if (i < q - 2 && j < q - 2 && k < q - 2) continue;
                double s = 0.0;
                for (int a = 0; a < q; ++a) s += Cm[i * q + a] * t2[(a * q + j) * q + k];
                eta += fabs(s);
            }
    free(t1);
    free(t2);
    return eta;
}

static int vbox_cmp_key(const void *a, const void *b)
{
    const vbox *x = (const vbox *)a, *y = (const vbox *)b;
    uint64_t kx = vkey(x->l, x->c), ky = vkey(y->l, y->c);
    if (kx != ky) return kx < ky ? -1 : 1;
    return x->l < y->l ? -1 : x->l > y->l;
}

/* does box (l, c) contain a feature point asking for a side below its own? */
static int feature_split(int l, const int32_t c[3], int nfeat, const double *feat)
{
    const double s = ldexp(1.0, -l);
    for (int f = 0; f < nfeat; ++f) {
        const double *F = feat + 4 * f;
        if (!(F[3] < s)) continue;
        int in = 1;
        for (int d = 0; d < 3; ++d) {
            double lo = -0.5 + c[d] * s, hi = lo + s;
            in &= (F[d] >= lo) && (F[d] < hi);
        }
        if (in) return 1;
    }
    return 0;
}

int orc_vtree_build(const orc_vparams *vp, double rho_scale, int minlevel, int maxlevel,
                    int nfeat, const double *feat, orc_density_fn fn, void *ctx, orc_vtree *t)
{
    memset(t, 0, sizeof(*t));
    const int q = vp->q, q3 = q * q * q;
    if (maxlevel < 0 || maxlevel > 19 || minlevel < 0 || minlevel > maxlevel) return -1;
    int64_t cap = 1024, nleaf = 0;
    vbox *leaves = (vbox *)malloc((size_t)cap * sizeof(vbox));
    vbox *cur = (vbox *)malloc(sizeof(vbox));
    int64_t ncur = 1;
    cur[0].l = 0;
    cur[0].c[0] = cur[0].c[1] = cur[0].c[2] = 0;
    /* refinement by resolution, level by level */
    for (int l = 0; ncur > 0; ++l) {
        uint8_t *split = (uint8_t *)calloc((size_t)ncur, 1);
        if (l < maxlevel) {
            double *xyz = (double *)malloc((size_t)ncur * q3 * 3 * sizeof(double));
            double *f = (double *)malloc((size_t)ncur * q3 * sizeof(double));
            for (int64_t b = 0; b < ncur; ++b)
                for (int i = 0; i < q; ++i)
                    for (int j = 0; j < q; ++j)
                        for (int k = 0; k < q; ++k)
                            node_coord(q, l, cur[b].c, i, j, k, &xyz[3 * (b * q3 + (i * q + j) * q + k)]);
            if (l >= minlevel) fn(ncur * q3, xyz, f, ctx);
            for (int64_t b = 0; b < ncur; ++b)
                split[b] = (l < minlevel) || feature_split(l, cur[b].c, nfeat, feat) ||
                           tail_coef(q, f + b * q3) > vp->tol * rho_scale;
            free(xyz);
            free(f);
        }
        int64_t nsplit = 0;
        for (int64_t b = 0; b < ncur; ++b) nsplit += split[b];
        vbox *nxt = (vbox *)malloc((size_t)(nsplit ? 8 * nsplit : 1) * sizeof(vbox));
        int64_t nn = 0;
        for (int64_t b = 0; b < ncur; ++b) {
            if (!split[b]) {
                if (nleaf == cap) { cap *= 2; leaves = (vbox *)realloc(leaves, (size_t)cap * sizeof(vbox)); }
                leaves[nleaf++] = cur[b];
                continue;
            }
            for (int o = 0; o < 8; ++o) {
                nxt[nn].l = l + 1;
                nxt[nn].c[0] = 2 * cur[b].c[0] + ((o >> 2) & 1);
                nxt[nn].c[1] = 2 * cur[b].c[1] + ((o >> 1) & 1);
                nxt[nn].c[2] = 2 * cur[b].c[2] + (o & 1);
                ++nn;
            }
        }
        free(split);
        free(cur);
        cur = nxt;
        ncur = nn;
    }
    free(cur);

    /* 2:1 balance: split any leaf that touches a leaf two or more levels finer */
    for (;;) {
        uint64_t *codes = (uint64_t *)malloc((size_t)nleaf * sizeof(uint64_t));
        for (int64_t i = 0; i < nleaf; ++i) codes[i] = vcode(leaves[i].l, leaves[i].c);
        qsort(codes, (size_t)nleaf, sizeof(uint64_t), u64cmp);
        uint64_t *mark = (uint64_t *)malloc((size_t)(nleaf ? nleaf : 1) * 26 * sizeof(uint64_t));
        int64_t nmark = 0;
        for (int64_t i = 0; i < nleaf; ++i) {
            const int b = leaves[i].l;
            if (b < 2) continue;
            const int32_t lim = 1 << b;
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        if (!dx && !dy && !dz) continue;
                        int32_t nc[3] = {leaves[i].c[0] + dx, leaves[i].c[1] + dy, leaves[i].c[2] + dz};
                        if (nc[0] < 0 || nc[1] < 0 || nc[2] < 0 || nc[0] >= lim || nc[1] >= lim || nc[2] >= lim)
                            continue;
                        for (int a = b; a >= 0; --a) {
                            int32_t ac[3] = {nc[0] >> (b - a), nc[1] >> (b - a), nc[2] >> (b - a)};
                            uint64_t cd = vcode(a, ac);
                            if (has_code(codes, nleaf, cd)) {
                                if (a <= b - 2) mark[nmark++] = cd;
                                break;
                            }
                        }
                    }
        }
        if (nmark == 0) {
            free(codes);
            free(mark);
            break;
        }
        qsort(mark, (size_t)nmark, sizeof(uint64_t), u64cmp);
        int64_t nu = 0;
        for (int64_t i = 0; i < nmark; ++i)
            if (nu == 0 || mark[nu - 1] != mark[i]) mark[nu++] = mark[i];
        vbox *nl = (vbox *)malloc((size_t)(nleaf + 7 * nu) * sizeof(vbox));
        int64_t m = 0;
        for (int64_t i = 0; i < nleaf; ++i) {
            if (!has_code(mark, nu, vcode(leaves[i].l, leaves[i].c))) {
                nl[m++] = leaves[i];
                continue;
            }
            for (int o = 0; o < 8; ++o) {
                nl[m].l = leaves[i].l + 1;
                nl[m].c[0] = 2 * leaves[i].c[0] + ((o >> 2) & 1);
                nl[m].c[1] = 2 * leaves[i].c[1] + ((o >> 1) & 1);
                nl[m].c[2] = 2 * leaves[i].c[2] + (o & 1);
                ++m;
            }
        }
        free(leaves);
        leaves = nl;
        nleaf = m;
        cap = m;
        free(codes);
        free(mark);
    }
    qsort(leaves, (size_t)nleaf, sizeof(vbox), vbox_cmp_key);
    t->q = q;
    t->nleaf = nleaf;
    t->level = (int32_t *)malloc((size_t)(nleaf ? nleaf : 1) * sizeof(int32_t));
    t->ijk = (int32_t *)malloc((size_t)(nleaf ? nleaf : 1) * 3 * sizeof(int32_t));
    for (int64_t i = 0; i < nleaf; ++i) {
        t->level[i] = leaves[i].l;
        for (int d = 0; d < 3; ++d) t->ijk[3 * i + d] = leaves[i].c[d];
    }
    free(leaves);
    return 0;
}

void orc_vtree_free(orc_vtree *t)
{
    free(t->level);
    free(t->ijk);
    memset(t, 0, sizeof(*t));
}

void orc_vol_nodes(const orc_vtree *t, double *xyz)
{
    const int q = t->q, q3 = q * q * q;
    for (int64_t b = 0; b < t->nleaf; ++b)
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < q; ++k)
                    node_coord(q, t->level[b], &t->ijk[3 * b], i, j, k, &xyz[3 * (b * q3 + (i * q + j) * q + k)]);
}

/* ---------------------------------------------------------- evaluation */
/* dense 3-index mode products t[i0][i1][i2] (dims n), axis k replaced by mo */
static void vmode(const double *in, const int n[3], int k, const double *M, int mo, double *out)
{
    int no[3] = {n[0], n[1], n[2]};
    no[k] = mo;
    for (int a = 0; a < no[0]; ++a)
        for (int b = 0; b < no[1]; ++b)
            for (int c = 0; c < no[2]; ++c) {
                int o[3] = {a, b, c};
                double s = 0.0;
                for (int j = 0; j < n[k]; ++j) {
                    int ii[3] = {a, b, c};
                    ii[k] = j;
                    s += M[o[k] * n[k] + j] * in[(ii[0] * n[1] + ii[1]) * n[2] + ii[2]];
                }
                out[(a * no[1] + b) * no[2] + c] = s;
            }
}

/* apply M0 (x), M1 (y), M2 (z), each (mo x ni), to in[ni^3] -> out[mo^3] */
static void vapply3(const double *in, int ni, const double *M0, const double *M1, const double *M2, int mo,
                    double *out)
{
    double *t1 = (double *)malloc((size_t)ni * ni * mo * sizeof(double));
    double *t2 = (double *)malloc((size_t)ni * mo * mo * sizeof(double));
    int d0[3] = {ni, ni, ni}, d1[3] = {ni, ni, mo}, d2[3] = {ni, mo, mo};
    vmode(in, d0, 2, M2, mo, t1);
    vmode(t1, d1, 1, M1, mo, t2);
    vmode(t2, d2, 0, M0, mo, out);
    free(t1);
    free(t2);
}

static void cmode(const cplx *in, const int n[3], int k, const cplx *M, int mo, cplx *out)
{
    int no[3] = {n[0], n[1], n[2]};
    no[k] = mo;
    for (int a = 0; a < no[0]; ++a)
        for (int b = 0; b < no[1]; ++b)
            for (int c = 0; c < no[2]; ++c) {
                int o[3] = {a, b, c};
                cplx s = 0.0;
                for (int j = 0; j < n[k]; ++j) {
                    int ii[3] = {a, b, c};
                    ii[k] = j;
                    s += M[o[k] * n[k] + j] * in[(ii[0] * n[1] + ii[1]) * n[2] + ii[2]];
                }
                out[(a * no[1] + b) * no[2] + c] = s;
            }
}

/* proxies -> plane waves Phi_m = sum_j exp(-i h m.(r_j - c)) rho_j */
static void v_proxy_to_pw(const cheb_t *ch, const double *rho, double h, double s, int nm, cplx *phi)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *E = (cplx *)malloc((size_t)n * p * sizeof(cplx));
    for (int m = 0; m < n; ++m)
        for (int j = 0; j < p; ++j) E[m * p + j] = cexp(-I * h * (m - nm) * 0.5 * s * ch->x[j]);
    cplx *t0 = (cplx *)malloc((size_t)p * p * p * sizeof(cplx));
    for (int i = 0; i < p * p * p; ++i) t0[i] = rho[i];
    int d0[3] = {p, p, p}, d1[3] = {p, p, n}, d2[3] = {p, n, n};
    cplx *t1 = (cplx *)malloc((size_t)p * p * n * sizeof(cplx));
    cplx *t2 = (cplx *)malloc((size_t)p * n * n * sizeof(cplx));
    cmode(t0, d0, 2, E, n, t1);
    cmode(t1, d1, 1, E, n, t2);
    cmode(t2, d2, 0, E, n, phi);
    free(E); free(t0); free(t1); free(t2);
}

/* incoming plane waves -> values on the Chebyshev grid, added to v */
static void v_pw_to_grid(const cheb_t *ch, const cplx *psi, double h, double s, int nm, double *v)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *G = (cplx *)malloc((size_t)p * n * sizeof(cplx));
    for (int j = 0; j < p; ++j)
        for (int m = 0; m < n; ++m) G[j * n + m] = cexp(I * h * (m - nm) * 0.5 * s * ch->x[j]);
    int d0[3] = {n, n, n}, d1[3] = {n, n, p}, d2[3] = {n, p, p};
    cplx *t1 = (cplx *)malloc((size_t)n * n * p * sizeof(cplx));
    cplx *t2 = (cplx *)malloc((size_t)n * p * p * sizeof(cplx));
    cplx *t3 = (cplx *)malloc((size_t)p * p * p * sizeof(cplx));
    cmode(psi, d0, 2, G, p, t1);
    cmode(t1, d1, 1, G, p, t2);
    cmode(t2, d2, 0, G, p, t3);
    for (int i = 0; i < p * p * p; ++i) v[i] += creal(t3[i]);
    free(G); free(t1); free(t2); free(t3);
}

typedef struct {
    int64_t nbox;
    int nlev;
    int64_t *lstart;   /* [nlev+1] boxes sorted by (level, Morton key) */
    vbox *b;
    uint64_t *code;    /* [nbox] vcode, ascending within a level and overall */
    int64_t *leafidx;  /* [nbox] leaf index or -1 */
    int64_t *child0;   /* [nbox] first child or -1 */
} vboxes;

static int64_t find_box(const vboxes *B, int l, const int32_t c[3])
{
    if (l >= B->nlev) return -1;
    int32_t lim = 1 << l;
    if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= lim || c[1] >= lim || c[2] >= lim) return -1;
    uint64_t v = vcode(l, c);
    int64_t lo = B->lstart[l], hi = B->lstart[l + 1];
    while (lo < hi) {
        int64_t m = (lo + hi) / 2;
        if (B->code[m] < v) lo = m + 1;
        else hi = m;
    }
    return (lo < B->lstart[l + 1] && B->code[lo] == v) ? lo : -1;
}

static int box_cmp_code(const void *a, const void *b)
{
    const vbox *x = (const vbox *)a, *y = (const vbox *)b;
    uint64_t cx = vcode(x->l, x->c), cy = vcode(y->l, y->c);
    return cx < cy ? -1 : cx > cy;
}

static void build_boxes(const orc_vtree *t, vboxes *B)
{
    int maxl = 0;
    for (int64_t i = 0; i < t->nleaf; ++i)
        if (t->level[i] > maxl) maxl = t->level[i];
    int64_t cap = t->nleaf * 2 + 16, n = 0;
    vbox *all = (vbox *)malloc((size_t)cap * sizeof(vbox));
    for (int64_t i = 0; i < t->nleaf; ++i)
        for (int a = t->level[i]; a >= 0; --a) {
            if (n == cap) { cap *= 2; all = (vbox *)realloc(all, (size_t)cap * sizeof(vbox)); }
            all[n].l = a;
            for (int d = 0; d < 3; ++d) all[n].c[d] = t->ijk[3 * i + d] >> (t->level[i] - a);
            ++n;
        }
    qsort(all, (size_t)n, sizeof(vbox), box_cmp_code);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (m == 0 || vcode(all[m - 1].l, all[m - 1].c) != vcode(all[i].l, all[i].c)) all[m++] = all[i];
    B->nbox = m;
    B->b = all;
    B->nlev = maxl + 1;
    B->lstart = (int64_t *)calloc((size_t)B->nlev + 1, sizeof(int64_t));
    B->code = (uint64_t *)malloc((size_t)m * sizeof(uint64_t));
    for (int64_t i = 0; i < m; ++i) {
        B->code[i] = vcode(all[i].l, all[i].c);
        B->lstart[all[i].l + 1]++;
    }
    for (int l = 0; l < B->nlev; ++l) B->lstart[l + 1] += B->lstart[l];
    B->leafidx = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    B->child0 = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) B->leafidx[i] = -1;
    for (int64_t i = 0; i < t->nleaf; ++i) {
        int32_t c[3] = {t->ijk[3 * i], t->ijk[3 * i + 1], t->ijk[3 * i + 2]};
        B->leafidx[find_box(B, t->level[i], c)] = i;
    }
    for (int64_t i = 0; i < m; ++i) {
        int32_t c[3] = {2 * all[i].c[0], 2 * all[i].c[1], 2 * all[i].c[2]};
        B->child0[i] = (B->leafidx[i] >= 0) ? -1 : find_box(B, all[i].l + 1, c);
    }
}

static void free_boxes(vboxes *B)
{
    free(B->lstart); free(B->b); free(B->code); free(B->leafidx); free(B->child0);
}

/* second-derivative matrix of the q-point Chebyshev interpolant on [-1,1] */
static void cheb_d2(const cheb_t *chq, double *D2)
{
    const int q = chq->p;
    for (int i = 0; i < q; ++i) {
        double x = chq->x[i];
        /* T_n''(x) from T_n'' = n ((n+1) T_n - U_n) / (x^2 - 1) */
        double T[32], U[32], Tpp[32];
        T[0] = 1.0; U[0] = 1.0;
        if (q > 1) { T[1] = x; U[1] = 2.0 * x; }
        for (int n = 2; n < q; ++n) {
            T[n] = 2.0 * x * T[n - 1] - T[n - 2];
            U[n] = 2.0 * x * U[n - 1] - U[n - 2];
        }
        for (int n = 0; n < q; ++n) Tpp[n] = (n < 2) ? 0.0 : n * ((n + 1) * T[n] - U[n]) / (x * x - 1.0);
        for (int j = 0; j < q; ++j) {
            double s = 0.0;
            for (int n = 0; n < q; ++n) s += Tpp[n] * chq->vinv[n * q + j];
            D2[i * q + j] = s;
        }
    }
}

/* Laplacian of the leaf polynomial at its nodes (leaf side s) */
static void leaf_laplacian(int q, const double *D2, double s, const double *f, double *out)
{
    const double sc = 4.0 / (s * s);
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int c = 0; c < q; ++c) {
                double v = 0.0;
                for (int j = 0; j < q; ++j) {
                    v += D2[a * q + j] * f[(j * q + b) * q + c];
                    v += D2[b * q + j] * f[(a * q + j) * q + c];
                    v += D2[c * q + j] * f[(a * q + b) * q + j];
                }
                out[(a * q + b) * q + c] = v * sc;
            }
}

int orc_vol_eval(const orc_vtree *t, const orc_vparams *vp, const double *rho, orc_vol_result *res)
{
    memset(res, 0, sizeof(*res));
    const int q = vp->q, q3 = q * q * q, p = vp->p, p3 = p * p * p;
    if (t->q != q || t->nleaf < 1) return -1;
    const int nf = vp->nf, nn = 2 * nf + 1, n3 = nn * nn * nn;
    const int nw = vp->nw, nwn = 2 * nw + 1, nw3 = nwn * nwn * nwn;
    const int64_t nleaf = t->nleaf, npt = nleaf * q3;
    res->n = npt;
    res->u = (double *)calloc((size_t)npt, sizeof(double));
    res->ufar = (double *)calloc((size_t)npt, sizeof(double));
    res->unear = (double *)calloc((size_t)npt, sizeof(double));
    res->utail = (double *)calloc((size_t)npt, sizeof(double));
    const double kappa = 1.0 / (4.0 * M_PI);

    orc_pswf ps; /* PSWF split (tol 1e-6): D_l and W_0 of Sec. 3.7 */
    if (vp->split == 1 && orc_pswf_init(vp->c, &ps) != 0) return -1;
    vboxes B;
    build_boxes(t, &B);
    cheb_t ch, chq;
    cheb_init(p, &ch);
    cheb_init(q, &chq);

    /* V[a][j] = int_{-1}^{1} ell_a(eta) L_j(eta) d eta by nleg-point Gauss-Legendre
       (proxy grid Lagrange basis ell_a, leaf grid Lagrange basis L_j) */
    double *V = (double *)calloc((size_t)p * q, sizeof(double));
    {
        double gx[64], gw[64], la[64], lj[64];
        orc_gauss_legendre(vp->nleg, gx, gw);
        for (int n = 0; n < vp->nleg; ++n) {
            cheb_interp_row(&ch, gx[n], la);
            cheb_interp_row(&chq, gx[n], lj);
            for (int a = 0; a < p; ++a)
                for (int j = 0; j < q; ++j) V[a * q + j] += gw[n] * la[a] * lj[j];
        }
    }
    /* U[i][a] = ell_a(x_i): proxy-grid polynomial at the leaf nodes */
    double *U = (double *)malloc((size_t)q * p * sizeof(double));
    for (int i = 0; i < q; ++i) cheb_interp_row(&ch, chq.x[i], &U[i * p]);

    double **proxy = (double **)calloc((size_t)B.nbox, sizeof(double *));
    double **local = (double **)calloc((size_t)B.nbox, sizeof(double *));

    /* ---- proxy charges: leaves from the density (Gauss-Legendre weights
       times rho at the Legendre nodes, anterpolated), parents by merging */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < B.nbox; ++b) {
        if (B.leafidx[b] < 0) continue;
        double s = ldexp(1.0, -B.b[b].l), sc = 0.125 * s * s * s;
        proxy[b] = (double *)malloc((size_t)p3 * sizeof(double));
        vapply3(rho + B.leafidx[b] * q3, q, V, V, V, p, proxy[b]);
        for (int i = 0; i < p3; ++i) proxy[b][i] *= sc;
    }
    for (int l = B.nlev - 2; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = B.lstart[l]; b < B.lstart[l + 1]; ++b) {
            if (B.leafidx[b] >= 0) continue;
            double *acc = (double *)calloc((size_t)p3, sizeof(double));
            double *tA = (double *)malloc((size_t)p3 * sizeof(double));
            for (int k = 0; k < 8; ++k) {
                int64_t c = B.child0[b] + k;
                vapply3(proxy[c], p, ch.A[(k >> 2) & 1], ch.A[(k >> 1) & 1], ch.A[k & 1], p, tA);
                for (int i = 0; i < p3; ++i) acc[i] += tA[i];
            }
            free(tA);
            proxy[b] = acc;
        }
    }

    /* ---- root: windowed kernel W_0 over the whole unit box */
    {
        const double hw = vp->hw, fac = pow(hw / (2.0 * M_PI), 3);
        cplx *phi = (cplx *)malloc((size_t)nw3 * sizeof(cplx));
        v_proxy_to_pw(&ch, proxy[0], hw, 1.0, nw, phi);
        for (int a = 0; a < nwn; ++a)
            for (int b = 0; b < nwn; ++b)
                for (int c = 0; c < nwn; ++c) {
                    int k2 = (a - nw) * (a - nw) + (b - nw) * (b - nw) + (c - nw) * (c - nw);
                    const double k = hw * sqrt((double)k2);
                    phi[(a * nwn + b) * nwn + c] *= fac * (vp->split ? orc_w0hat(&ps, k) : orc_gw0hat(vp, k));
                }
        local[0] = (double *)calloc((size_t)p3, sizeof(double));
        v_pw_to_grid(&ch, phi, hw, 1.0, nw, local[0]);
        free(phi);
    }

    /* ---- downward pass: D_l between colleagues (F_out = non-leaf source
       boxes), local values split to children, leaves evaluated on their grid */
    cplx **phi = (cplx **)calloc((size_t)B.nbox, sizeof(cplx *));
    for (int l = 0; l < B.nlev; ++l) {
        const int64_t b0 = B.lstart[l], b1 = B.lstart[l + 1];
        const double s = ldexp(1.0, -l), h = 2.0 * M_PI / (3.0 * s), fac = pow(h / (2.0 * M_PI), 3);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (B.leafidx[b] >= 0) continue;
            phi[b] = (cplx *)malloc((size_t)n3 * sizeof(cplx));
            v_proxy_to_pw(&ch, proxy[b], h, s, nf, phi[b]);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            cplx *psi = NULL;
            for (int k = 0; k < 27; ++k) {
                int d[3] = {k / 9 - 1, (k / 3) % 3 - 1, k % 3 - 1};
                int32_t nc[3] = {B.b[b].c[0] + d[0], B.b[b].c[1] + d[1], B.b[b].c[2] + d[2]};
                int64_t sb = find_box(&B, l, nc);
                if (sb < 0 || B.leafidx[sb] >= 0) continue;
                if (!psi) psi = (cplx *)calloc((size_t)n3, sizeof(cplx));
                cplx e0[64], e1[64], e2[64];
                for (int m = 0; m < nn; ++m) {
                    /* exp(i h m (c_B - c_S)), c_B - c_S = -d s */
                    e0[m] = cexp(-I * h * (m - nf) * d[0] * s);
                    e1[m] = cexp(-I * h * (m - nf) * d[1] * s);
                    e2[m] = cexp(-I * h * (m - nf) * d[2] * s);
                }
                for (int a = 0; a < nn; ++a)
                    for (int bb = 0; bb < nn; ++bb)
                        for (int cc = 0; cc < nn; ++cc) {
                            int idx = (a * nn + bb) * nn + cc;
                            psi[idx] += e0[a] * e1[bb] * e2[cc] * phi[sb][idx];
                        }
            }
            if (!local[b]) local[b] = (double *)calloc((size_t)p3, sizeof(double));
            if (!psi) continue;
            for (int a = 0; a < nn; ++a)
                for (int bb = 0; bb < nn; ++bb)
                    for (int cc = 0; cc < nn; ++cc) {
                        int k2 = (a - nf) * (a - nf) + (bb - nf) * (bb - nf) + (cc - nf) * (cc - nf);
                        const double k = h * sqrt((double)k2);
                        psi[(a * nn + bb) * nn + cc] *= fac * (vp->split ? orc_dhat(&ps, l, k) : orc_gdhat(vp, l, k));
                    }
            v_pw_to_grid(&ch, psi, h, s, nf, local[b]);
            free(psi);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (B.leafidx[b] >= 0) {
                double *out = res->ufar + B.leafidx[b] * q3;
                vapply3(local[b], p, U, U, U, q, out);
                continue;
            }
            double *AT[2];
            for (int sg = 0; sg < 2; ++sg) {
                AT[sg] = (double *)malloc((size_t)p * p * sizeof(double));
                for (int i = 0; i < p; ++i)
                    for (int a = 0; a < p; ++a) AT[sg][i * p + a] = ch.A[sg][a * p + i];
            }
            for (int k = 0; k < 8; ++k) {
                int64_t c = B.child0[b] + k;
                local[c] = (double *)malloc((size_t)p3 * sizeof(double));
                vapply3(local[b], p, AT[(k >> 2) & 1], AT[(k >> 1) & 1], AT[k & 1], p, local[c]);
            }
            free(AT[0]);
            free(AT[1]);
        }
        for (int64_t b = b0; b < b1; ++b) {
            free(phi[b]); phi[b] = NULL;
            free(local[b]); local[b] = NULL;
        }
    }
    free(phi);

    /* ---- near field: for each source leaf T, the Gaussians of R_{L_T} with
       t in [1/sigma_{L_T}, t_a(target)] (PSWF split: [theta1/s_T, t_a] and
       the fitted Gaussians) over the target leaves of its lists */
    const double sqL = sqrt(log(1.0 / vp->tol));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t T = 0; T < B.nbox; ++T) {
        if (B.leafidx[T] < 0) continue;
        const int L = B.b[T].l;
        const double sT = ldexp(1.0, -L);
        double cT[3];
        for (int d = 0; d < 3; ++d) cT[d] = -0.5 + (B.b[T].c[d] + 0.5) * sT;
        /* target leaves: leaves in the colleagues' subtrees, coarse-neighbour leaves */
        int64_t *tg = NULL;
        int64_t ntg = 0, cap = 0;
        for (int k = 0; k < 27; ++k) {
            int32_t nc[3] = {B.b[T].c[0] + k / 9 - 1, B.b[T].c[1] + (k / 3) % 3 - 1, B.b[T].c[2] + k % 3 - 1};
            int32_t lim = 1 << L;
            if (nc[0] < 0 || nc[1] < 0 || nc[2] < 0 || nc[0] >= lim || nc[1] >= lim || nc[2] >= lim) continue;
            int64_t cb = find_box(&B, L, nc);
            if (cb >= 0) {
                /* all leaves of the subtree of cb: a stack walk */
                int64_t stack[1024];
                int ns = 0;
                stack[ns++] = cb;
                while (ns) {
                    int64_t x = stack[--ns];
                    if (B.leafidx[x] >= 0) {
                        if (ntg == cap) { cap = cap ? 2 * cap : 64; tg = (int64_t *)realloc(tg, (size_t)cap * sizeof(int64_t)); }
                        tg[ntg++] = x;
                    } else {
                        for (int o = 0; o < 8; ++o) stack[ns++] = B.child0[x] + o;
                    }
                }
            } else if (L > 0) {
                int32_t pc[3] = {nc[0] >> 1, nc[1] >> 1, nc[2] >> 1};
                int64_t cb2 = find_box(&B, L - 1, pc);
                if (cb2 >= 0 && B.leafidx[cb2] >= 0) {
                    int dup = 0;
                    for (int64_t i = 0; i < ntg; ++i) dup |= (tg[i] == cb2);
                    if (!dup) {
                        if (ntg == cap) { cap = cap ? 2 * cap : 64; tg = (int64_t *)realloc(tg, (size_t)cap * sizeof(int64_t)); }
                        tg[ntg++] = cb2;
                    }
                }
            }
        }
        double tn[512], wn[512];
        double *G[3];
        for (int d = 0; d < 3; ++d) G[d] = (double *)malloc((size_t)q * q * sizeof(double));
        double *part = (double *)malloc((size_t)q3 * sizeof(double));
        const double *rT = rho + B.leafidx[T] * q3;
        for (int64_t it = 0; it < ntg; ++it) {
            const int64_t Bx = tg[it];
            const int LB = B.b[Bx].l;
            const double sB = ldexp(1.0, -LB);
            double cB[3], gap2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                cB[d] = -0.5 + (B.b[Bx].c[d] + 0.5) * sB;
                double g = fabs(cB[d] - cT[d]) - 0.5 * (sB + sT);
                if (g > 0.0) gap2 += g * g;
            }
            if (gap2 >= sT * sT) continue;
            const double t_lo = (vp->split ? vp->theta1 : sqL) / sT;
            int ng = orc_vsog(vp, t_lo, vp->tau_a / sB, tn, wn);
            for (int i = 0; i < vp->nfit; ++i, ++ng) { /* PSWF split: the fitted part of R_L */
                tn[ng] = vp->fit_t[i] / sT;
                wn[ng] = vp->fit_w[i] / sT;
            }
            double *ub = res->unear + B.leafidx[Bx] * q3;
            double row[16];
            for (int j = 0; j < ng; ++j) {
                const double tau = tn[j] * 0.5 * sT;
                for (int d = 0; d < 3; ++d)
                    for (int a = 0; a < q; ++a) {
                        double xa = cB[d] + 0.5 * sB * chq.x[a];
                        orc_vgauss_row(&chq, 2.0 * (xa - cT[d]) / sT, tau, row);
                        for (int bq = 0; bq < q; ++bq) G[d][a * q + bq] = 0.5 * sT * row[bq];
                    }
                vapply3(rT, q, G[0], G[1], G[2], q, part);
#pragma omp critical
                for (int i = 0; i < q3; ++i) ub[i] += wn[j] * part[i];
            }
        }
        for (int d = 0; d < 3; ++d) free(G[d]);
        free(part);
        free(tg);
    }

    /* ---- asymptotic part: Gaussians with t >= t_a(B) over R^3 from the
       target leaf's polynomial:  2 pi [rho/(2 t^2) + Lap rho/(16 t^4) +
       Lap^2 rho/(192 t^6)] */
    double *D2 = (double *)malloc((size_t)q * q * sizeof(double));
    cheb_d2(&chq, D2);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nleaf; ++i) {
        const double s = ldexp(1.0, -t->level[i]), ta = vp->tau_a / s;
        const double *f = rho + i * q3;
        double *l1 = (double *)malloc((size_t)q3 * sizeof(double)), *l2 = (double *)malloc((size_t)q3 * sizeof(double));
        leaf_laplacian(q, D2, s, f, l1);
        leaf_laplacian(q, D2, s, l1, l2);
        for (int k = 0; k < q3; ++k)
            res->utail[i * q3 + k] = 2.0 * M_PI * (f[k] / (2.0 * ta * ta) + l1[k] / (16.0 * pow(ta, 4)) +
                                                   l2[k] / (192.0 * pow(ta, 6)));
        free(l1);
        free(l2);
    }
    free(D2);

    for (int64_t i = 0; i < npt; ++i) {
        res->ufar[i] *= kappa;
        res->unear[i] *= kappa;
        res->utail[i] *= kappa;
        res->u[i] = res->ufar[i] + res->unear[i] + res->utail[i];
    }
    for (int64_t b = 0; b < B.nbox; ++b) free(proxy[b]);
    free(proxy);
    free(local);
    free(V);
    free(U);
    cheb_free(&ch);
    cheb_free(&chq);
    free_boxes(&B);
    return 0;
}

void orc_vol_result_free(orc_vol_result *r)
{
    free(r->u); free(r->ufar); free(r->unear); free(r->utail);
    memset(r, 0, sizeof(*r));
}
