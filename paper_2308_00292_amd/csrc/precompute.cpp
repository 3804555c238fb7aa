// Step 1 of the discrete DMK algorithm (Sec. 3.5): host-side precomputation
// in FP64 of everything the device stages read.
//
//  * psi_0^c, the first prolate spheroidal wave function of order zero
//    (Appendix, eigenfunction of F_c).  Its even Legendre coefficients are the
//    ground state of the prolate Sturm-Liouville operator, a symmetric matrix
//    in the normalised Legendre basis, diagonalised here by cyclic Jacobi
//    rotations.  Off [-1,1] psi is continued through the eigen-relation,
//    lambda_0 psi(x) = int_{-1}^1 psi(t) e^{icxt} dt, which in the Legendre
//    basis is a series of spherical Bessel functions:
//        int_{-1}^1 P_k(t) e^{iwt} dt = 2 i^k j_k(w).
//  * The cumulative window Phi(x) = (1/c_0) int_0^x psi (Sec. 3.7), tabulated
//    as Chebyshev coefficients of g(t) = Phi(sqrt t)/sqrt t on t in [0,1], so
//    that the residual kernel is R_l(r) = 1/r - g(r^2/s_l^2)/s_l for r < s_l.
//  * Plane-wave weights of the difference kernels (eq. differencekernelft3,
//    trapezoidal rule with spacing h_l = 2 pi/(3 s_l) and factor (h_l/2pi)^3)
//    and of the windowed root kernel (mollifier transform times the
//    transform 8 pi sin^2(kA/2)/k^2 of 1/r truncated at A = 1 + sqrt 3).
//  * 1-D operators: first-kind Chebyshev nodes, barycentric weights, the
//    child<->parent interpolation matrices of Lemmas 2.1/2.2 and the
//    proxy->plane-wave matrices of eq. outgoingexpansion2.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "dmk_internal.h"

namespace dmk {

bool params_for(double tol, Params *out, int dim)
{
    // Table 1 (c, N_1 = 2 nf + 1, p) plus a 1e-5 row (c = log(1/eps)).
    struct Row { double tol, c; int nf, p; };
    static const Row rows[] = {
        {1e-3, 7.2462000846862793, 6, 9},
        {1e-5, 11.512925464970229, 10, 15},
        {1e-6, 13.739999771118164, 12, 18},
        {1e-9, 20.736000061035156, 19, 28},
        {1e-12, 27.870000839233398, 26, 38},
    };
    for (const Row &r : rows) {
        if (std::fabs(std::log10(tol) - std::log10(r.tol)) < 1e-3) {
            out->tol = tol;
            out->c = r.c;
            out->nf = r.nf;
            out->p = r.p;
            // W_0 lives on r <= A + 1 (A = 1 + sqrt d); offsets inside the unit
            // box are <= 1 per axis, so the period 2 pi/hw must reach 3 + sqrt d.
            out->hw = 2.0 * M_PI / (3.0 + std::sqrt((double)dim));
            out->nw = (int)std::ceil(out->c / out->hw);
            return true;
        }
    }
    return false;
}

namespace {

// Cyclic Jacobi diagonalisation of a symmetric n x n matrix A (row-major,
// destroyed).  On return evals[i] and column i of V are an eigenpair.
void jacobi_eigen(int n, std::vector<double> &A, std::vector<double> &V, std::vector<double> &evals)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double a = A[(size_t)i * n + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    evals.resize(n);
    for (int i = 0; i < n; ++i) evals[i] = A[(size_t)i * n + i];
}

void legendre(int kmax, double x, std::vector<double> &P)
{
    P.resize(kmax + 1);
    P[0] = 1.0;
    if (kmax > 0) P[1] = x;
    for (int k = 1; k < kmax; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

// Spherical Bessel j_0..j_nmax at z > 0 by Miller's downward recurrence,
// normalised with j_0 or j_1 in closed form.
void sph_bessel(int nmax, double z, std::vector<double> &j)
{
    j.assign(nmax + 1, 0.0);
    if (z == 0.0) { j[0] = 1.0; return; }
    int N = nmax + 30 + (int)z;
    std::vector<double> v(N + 2, 0.0);
    double hi = 0.0, cur = 1e-280;
    for (int k = N; k >= 0; --k) {
        v[k] = cur;
        double lo = (2.0 * k + 1.0) / z * cur - hi;
        hi = cur;
        cur = lo;
        if (std::fabs(cur) > 1e200) {
            for (int m = k; m <= N; ++m) v[m] *= 1e-200;
            hi *= 1e-200;
            cur *= 1e-200;
        }
    }
    double j0 = std::sin(z) / z, j1 = std::sin(z) / (z * z) - std::cos(z) / z;
    double scale = (std::fabs(j0) >= std::fabs(j1)) ? j0 / v[0] : j1 / v[1];
    for (int k = 0; k <= nmax; ++k) j[k] = v[k] * scale;
}

double pswf_series(const Tables &t, double x)
{
    int K = (int)t.coef.size();
    std::vector<double> P;
    legendre(2 * K, x, P);
    double s = 0.0;
    for (int i = 0; i < K; ++i) s += t.coef[i] * std::sqrt(2 * i + 0.5) * P[2 * i];
    return s;
}

// Phi(x) = (1/c_0) int_0^x psi for 0 <= x <= 1 (Legendre antiderivatives).
double phi_window(const Tables &t, double x)
{
    if (x >= 1.0) return 1.0;
    int K = (int)t.coef.size();
    std::vector<double> P;
    legendre(2 * K + 1, x, P);
    double s = t.coef[0] * std::sqrt(0.5) * x;
    for (int i = 1; i < K; ++i) {
        int k = 2 * i;
        s += t.coef[i] * std::sqrt(k + 0.5) * (P[k + 1] - P[k - 1]) / (2.0 * k + 1.0);
    }
    return s / t.c0;
}

// Lagrange basis of the p first-kind Chebyshev nodes at xi (barycentric form).
void lagrange_row(const Tables &t, double xi, double *out)
{
    int p = t.p;
    for (int a = 0; a < p; ++a)
        if (xi == t.xcheb[a]) {
            for (int b = 0; b < p; ++b) out[b] = (a == b) ? 1.0 : 0.0;
            return;
        }
    double den = 0.0;
    for (int a = 0; a < p; ++a) {
        out[a] = t.bary[a] / (xi - t.xcheb[a]);
        den += out[a];
    }
    for (int a = 0; a < p; ++a) out[a] /= den;
}

}  // namespace

double pswf_phi(const Tables &t, double x) { return x <= 0.0 ? 0.0 : phi_window(t, x); }

double pswf_eval(const Tables &t, double x)
{
    x = std::fabs(x);
    if (x <= 1.0) return pswf_series(t, x);
    // psi(x) = (2/lambda_0) sum_i coef_i sqrt(k+1/2) (-1)^i j_k(c x), k = 2i
    int K = (int)t.coef.size();
    std::vector<double> j;
    sph_bessel(2 * K, t.prm.c * x, j);
    double s = 0.0;
    for (int i = 0; i < K; ++i) s += t.coef[i] * std::sqrt(2 * i + 0.5) * ((i & 1) ? -1.0 : 1.0) * j[2 * i];
    return 2.0 * s / t.lambda0;
}

void build_tables2(Tables *t);
void build_tables_pow2(Tables *t);

void build_tables(const Params &prm, Tables *t, int dim, int kind)
{
    t->kind = kind;
    t->prm = prm;
    t->dim = dim;
    const double c = prm.c;
    // ---- PSWF ground state in the even normalised-Legendre basis
    const int K = 48;
    std::vector<double> A((size_t)K * K, 0.0), V, ev;
    for (int i = 0; i < K; ++i) {
        double k = 2.0 * i;
        A[(size_t)i * K + i] = k * (k + 1.0) + c * c * (2.0 * k * k + 2.0 * k - 1.0) / ((2.0 * k - 1.0) * (2.0 * k + 3.0));
        if (i + 1 < K) {
            double off = c * c * (k + 1.0) * (k + 2.0) / ((2.0 * k + 3.0) * std::sqrt((2.0 * k + 1.0) * (2.0 * k + 5.0)));
            A[(size_t)i * K + i + 1] = off;
            A[(size_t)(i + 1) * K + i] = off;
        }
    }
    jacobi_eigen(K, A, V, ev);
    int imin = (int)(std::min_element(ev.begin(), ev.end()) - ev.begin());
    t->coef.resize(K);
    for (int i = 0; i < K; ++i) t->coef[i] = V[(size_t)i * K + imin];
    // trim negligible tail, fix the sign so that psi(0) > 0
    int keep = K;
    double cmax = 0.0;
    for (double v : t->coef) cmax = std::max(cmax, std::fabs(v));
    while (keep > 1 && std::fabs(t->coef[keep - 1]) < 1e-20 * cmax) keep--;
    t->coef.resize(keep);
    if (pswf_series(*t, 0.0) < 0)
        for (double &v : t->coef) v = -v;
    t->psi0 = pswf_series(*t, 0.0);
    // int_0^1 sqrt(k+1/2) P_k: sqrt(1/2) for k = 0, 0 for even k >= 2;
    // int_0^1 x^2 sqrt(k+1/2) P_k: sqrt(1/2)/3 (k = 0), 2 sqrt(5/2)/15 (k = 2).
    t->c0 = t->coef[0] * std::sqrt(0.5);
    t->c2 = t->coef[0] * std::sqrt(0.5) / 3.0 + (keep > 1 ? t->coef[1] * std::sqrt(2.5) * 2.0 / 15.0 : 0.0);
    t->lambda0 = 2.0 * t->c0 / t->psi0;

    // ---- sizes
    t->p = prm.p;
    t->nf = prm.nf;
    t->nn = 2 * prm.nf + 1;
    t->nh = prm.nf + 1;
    t->nw = prm.nw;
    t->nwn = 2 * prm.nw + 1;
    t->nwh = prm.nw + 1;
    const int p = t->p;

    // ---- Chebyshev nodes, barycentric weights, child<->parent matrices
    t->xcheb.resize(p);
    t->bary.resize(p);
    for (int j = 0; j < p; ++j) {
        t->xcheb[j] = std::cos(M_PI * (j + 0.5) / p);
        t->bary[j] = ((j & 1) ? -1.0 : 1.0) * std::sin((2 * j + 1) * M_PI / (2.0 * p));
    }
    t->c2p.assign((size_t)2 * p * p, 0.0);
    std::vector<double> row(p);
    for (int s = 0; s < 2; ++s) {
        double sigma = s ? 1.0 : -1.0;
        for (int i = 0; i < p; ++i) {
            lagrange_row(*t, 0.5 * (t->xcheb[i] + sigma), row.data());
            for (int a = 0; a < p; ++a) t->c2p[((size_t)s * p + a) * p + i] = row[a];
        }
    }
    // ---- proxy -> plane-wave matrices (complex, interleaved)
    t->epw.assign((size_t)t->nn * p * 2, 0.0);
    for (int m = -prm.nf; m <= prm.nf; ++m)
        for (int j = 0; j < p; ++j) {
            double ph = -M_PI * m * t->xcheb[j] / 3.0;
            t->epw[((size_t)(m + prm.nf) * p + j) * 2 + 0] = std::cos(ph);
            t->epw[((size_t)(m + prm.nf) * p + j) * 2 + 1] = std::sin(ph);
        }
    t->ew.assign((size_t)t->nwn * p * 2, 0.0);
    for (int m = -prm.nw; m <= prm.nw; ++m)
        for (int j = 0; j < p; ++j) {
            double ph = -prm.hw * m * 0.5 * t->xcheb[j];
            t->ew[((size_t)(m + prm.nw) * p + j) * 2 + 0] = std::cos(ph);
            t->ew[((size_t)(m + prm.nw) * p + j) * 2 + 1] = std::sin(ph);
        }

    if (dim == 2) {
        build_tables2(t);
        return;
    }
    if (kind == 2) {
        build_tables_pow2(t);
        return;
    }
    // ---- plane-wave weights of D_0 (level l multiplies by 2^l), half spectrum
    // w_0(m) = [psi(pi|m|/(3c)) - psi(2pi|m|/(3c))] / (3 pi psi(0) |m|^2),
    // w_0(0) = pi c_2 / (18 c_0)
    {
        int maxk2 = 3 * prm.nf * prm.nf;
        std::vector<double> memo(maxk2 + 1);
        memo[0] = M_PI * t->c2 / (18.0 * t->c0);
        for (int k2 = 1; k2 <= maxk2; ++k2) {
            double km = std::sqrt((double)k2);
            memo[k2] = (pswf_eval(*t, M_PI * km / (3.0 * c)) - pswf_eval(*t, 2.0 * M_PI * km / (3.0 * c))) /
                       (3.0 * M_PI * t->psi0 * k2);
        }
        // same layout as the plane-wave arrays: [m1][m3][m2]
        t->wd0.assign((size_t)t->nh * t->nn * t->nn, 0.0);
        for (int m1 = -prm.nf; m1 <= prm.nf; ++m1)
            for (int m3 = 0; m3 <= prm.nf; ++m3)
                for (int m2 = -prm.nf; m2 <= prm.nf; ++m2)
                    t->wd0[((size_t)(m1 + prm.nf) * t->nh + m3) * t->nn + (m2 + prm.nf)] =
                        memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
    // ---- windowed W_0 weights (hw/2pi)^3 * What_0(hw |m|)
    {
        const double Atr = 1.0 + std::sqrt(3.0);
        const double h = prm.hw, fac = std::pow(h / (2.0 * M_PI), 3);
        int maxk2 = 3 * prm.nw * prm.nw;
        std::vector<double> memo(maxk2 + 1);
        memo[0] = fac * 2.0 * M_PI * Atr * Atr;
        for (int k2 = 1; k2 <= maxk2; ++k2) {
            double k = h * std::sqrt((double)k2);
            double sn = std::sin(0.5 * k * Atr);
            memo[k2] = fac * 8.0 * M_PI * sn * sn / (k * k) * pswf_eval(*t, k / c) / t->psi0;
        }
        t->ww.assign((size_t)t->nwh * t->nwn * t->nwn, 0.0);
        for (int m3 = 0; m3 <= prm.nw; ++m3)
            for (int m2 = -prm.nw; m2 <= prm.nw; ++m2)
                for (int m1 = -prm.nw; m1 <= prm.nw; ++m1)
                    t->ww[((size_t)m3 * t->nwn + (m2 + prm.nw)) * t->nwn + (m1 + prm.nw)] =
                        memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
    // ---- residual window: Chebyshev coefficients of g(t) = Phi(sqrt t)/sqrt t
    {
        const int M = 48;
        std::vector<double> f(M), cf(M);
        for (int k = 0; k < M; ++k) {
            double u = std::cos(M_PI * (k + 0.5) / M);  // node in [-1,1]
            double tt = 0.5 * (u + 1.0);                 // t in [0,1]
            double x = std::sqrt(tt);
            f[k] = (x > 0) ? phi_window(*t, x) / x : t->psi0 / t->c0;
        }
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k) s += f[k] * std::cos(M_PI * j * (k + 0.5) / M);
            cf[j] = (j == 0 ? 1.0 : 2.0) * s / M;
        }
        // keep the terms above the rounding floor of the samples (~1e-15)
        int deg = M - 1;
        while (deg > 0 && std::fabs(cf[deg]) < 1e-14 * std::fabs(cf[0])) deg--;
        t->gdeg = deg;
        t->gcheb.assign(cf.begin(), cf.begin() + deg + 1);
        // FP32 evaluation needs only the terms above single-precision rounding
        int deg32 = deg;
        while (deg32 > 0 && std::fabs(cf[deg32]) < 1e-7 * std::fabs(cf[0])) deg32--;
        t->gdeg32 = deg32;
    }
}

// ---------------------------------------------------------------- 2-D
// Kernel -log(r)/(2 pi), split in Fourier space (Sec. 4.6): its transform
// 1/k^2 times the mollifier psi(k s_l/c)/psi(0).
//  * D_l weights (h_l/2pi)^2 Dhat_l(h_l |m|), h_l s_l = 2 pi/3:
//      w(m) = [psi(pi|m|/(3c)) - psi(2pi|m|/(3c))] / (4 pi^2 psi(0) |m|^2),
//      w(0) = c_2/(24 c_0) (the k -> 0 limit), the same at every level
//      (scale invariance of the log kernel up to a constant).
//  * W_0 weights (hw/2pi)^2 psi(k/c)/psi(0) That(k), That the transform of the
//    kernel cut at A = 1 + sqrt 2 (Sec. 4.7):
//      That(k) = (1 - J_0(kA))/k^2 - A log(A) J_1(kA)/k, That(0) = A^2/4 - A^2 log(A)/2.
//  * The residual R_l(r) = -log(x)/(2 pi) - m(x), x = r/s_l < 1, with
//      m(x) = (1/2 pi) int_0^{2c} psi(t/c)/psi(0) (J_0(tx) - J_0(t)) dt/t
//    (the mollifier beyond argument 2 is dropped), tabulated as a Chebyshev
//    series in u = 2x^2 - 1 from values by Gauss-Legendre quadrature on
//    uniform panels.
void build_tables2(Tables *t)
{
    const Params &prm = t->prm;
    const double c = prm.c;
    {
        const int nf = prm.nf, nn = t->nn, nh = t->nh;
        const int maxk2 = 2 * nf * nf;
        std::vector<double> memo(maxk2 + 1);
        memo[0] = t->c2 / (24.0 * t->c0);
        for (int k2 = 1; k2 <= maxk2; ++k2) {
            double km = std::sqrt((double)k2);
            memo[k2] = (pswf_eval(*t, M_PI * km / (3.0 * c)) - pswf_eval(*t, 2.0 * M_PI * km / (3.0 * c))) /
                       (4.0 * M_PI * M_PI * t->psi0 * k2);
        }
        t->wd0.assign((size_t)nn * nh, 0.0);
        for (int m1 = -nf; m1 <= nf; ++m1)
            for (int m2 = 0; m2 <= nf; ++m2) t->wd0[(size_t)(m1 + nf) * nh + m2] = memo[m1 * m1 + m2 * m2];
    }
    {
        const int nw = prm.nw, nwn = t->nwn, nwh = t->nwh;
        const double Atr = 1.0 + std::sqrt(2.0), h = prm.hw, fac = std::pow(h / (2.0 * M_PI), 2);
        const int maxk2 = 2 * nw * nw;
        std::vector<double> memo(maxk2 + 1);
        memo[0] = fac * (0.25 * Atr * Atr - 0.5 * Atr * Atr * std::log(Atr));
        for (int k2 = 1; k2 <= maxk2; ++k2) {
            double k = h * std::sqrt((double)k2);
            double That = (1.0 - std::cyl_bessel_j(0.0, k * Atr)) / (k * k) -
                          Atr * std::log(Atr) * std::cyl_bessel_j(1.0, k * Atr) / k;
            memo[k2] = fac * That * pswf_eval(*t, k / c) / t->psi0;
        }
        t->ww.assign((size_t)nwn * nwh, 0.0);
        for (int m1 = -nw; m1 <= nw; ++m1)
            for (int m2 = 0; m2 <= nw; ++m2) t->ww[(size_t)(m1 + nw) * nwh + m2] = memo[m1 * m1 + m2 * m2];
    }
    {
        // quadrature nodes on [0, 2c]: 24 uniform panels of 32 Gauss-Legendre points
        const int NPAN = 24, NG = 32;
        std::vector<double> gx(NG), gw(NG);
        for (int i = 0; i < NG; ++i) {  // Newton on P_NG
            double z = std::cos(M_PI * (i + 0.75) / (NG + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= NG; ++k) {
                    double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = pk;
                }
                double dp = NG * (z * p1 - p0) / (z * z - 1.0);
                double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) {
                    gw[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                    break;
                }
                gw[i] = 2.0 / ((1.0 - z * z) * dp * dp);
            }
            gx[i] = z;
        }
        const double T = 2.0 * c, hp = T / NPAN;
        std::vector<double> tq, wq;
        for (int pnl = 0; pnl < NPAN; ++pnl)
            for (int i = 0; i < NG; ++i) {
                double tt = hp * (pnl + 0.5 * (gx[i] + 1.0));
                tq.push_back(tt);
                wq.push_back(0.5 * hp * gw[i] * pswf_eval(*t, tt / c) / t->psi0 / tt / (2.0 * M_PI));
            }
        auto mval = [&](double x) {
            double s = 0.0;
            for (size_t k = 0; k < tq.size(); ++k)
                s += wq[k] * (std::cyl_bessel_j(0.0, tq[k] * x) - std::cyl_bessel_j(0.0, tq[k]));
            return s;
        };
        const int M = 48;
        std::vector<double> f(M), cf(M);
        for (int k = 0; k < M; ++k) {
            double u = std::cos(M_PI * (k + 0.5) / M);
            f[k] = mval(std::sqrt(0.5 * (u + 1.0)));
        }
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k) s += f[k] * std::cos(M_PI * j * (k + 0.5) / M);
            cf[j] = (j == 0 ? 1.0 : 2.0) * s / M;
        }
        double cmax = 0.0;
        for (double v : cf) cmax = std::max(cmax, std::fabs(v));
        // keep the terms above the rounding floor of the samples (~2e-15 of
        // the largest coefficient)
        int deg = M - 1;
        while (deg > 0 && std::fabs(cf[deg]) < 1e-14 * cmax) deg--;
        t->gdeg = deg;
        t->gcheb.assign(cf.begin(), cf.begin() + deg + 1);
        int deg32 = deg;
        while (deg32 > 0 && std::fabs(cf[deg32]) < 1e-8 * cmax) deg32--;
        t->gdeg32 = deg32;
        t->m0 = mval(0.0);
    }
}


// ---------------------------------------------------------------- 1/r^2
// Kernel 1/r^2 in 3-D with the PSWF power-function split (Sec. 4.5, alpha = 2):
//   Phi2(x) = (1/C_1) int_0^x t psi(t) dt (x <= 1; 1 beyond), C_1 = int_0^1 t psi,
//   D_l(r) = (Phi2(r/s_{l+1}) - Phi2(r/s_l))/r^2 = 4^l D_0(2^l r),
//   R_L(r) = (1 - Phi2(r/s_L))/r^2 = 1/r^2 - g2(r^2/s_L^2)/s_L^2 for r < s_L,
// with g2(t) = Phi2(sqrt t)/t smooth on [0, 1] (g2(0) = psi(0)/(2 C_1), the
// self term).  Phi2 from Legendre integrals of the PSWF's series:
// t P_n = ((n+1) P_{n+1} + n P_{n-1})/(2n+1), int_0^x P_m = (P_{m+1} - P_{m-1})/(2m+1) |_0^x.
//  * level-0 weights (h_0/2pi)^3 Dhat_0(h_0 |m|), Dhat_0(k) = (4 pi/k) int_0^1 D_0(r) r sin(kr) dr
//    (Gauss-Legendre panels on [0, 1/2] and [1/2, 1]); level l multiplies by 4^l;
//  * root: W_0 = M_0 chi with M_0 = Phi2(r)/r^2 and chi a smooth step from 1
//    at sqrt 3 to 0 at sqrt 3 + 2, chi = (1 - sign(y) Phi(|y|))/2, y = r - sqrt 3 - 1,
//    Phi the 1/r split's window; its transform by radial quadrature;
//  * residual series: g2 as a Chebyshev series in 2t - 1.
namespace {

double phi2_raw(const Tables &t, double x)  // int_0^x t psi(t) dt
{
    const int K = (int)t.coef.size(), kmax = 2 * K + 2;
    std::vector<double> Px, P0;
    legendre(kmax, x, Px);
    legendre(kmax, 0.0, P0);
    auto I = [&](int m) {  // int_0^x P_m
        if (m == 0) return x;
        return (Px[m + 1] - Px[m - 1] - P0[m + 1] + P0[m - 1]) / (2.0 * m + 1.0);
    };
    double s = 0.0;
    for (int i = 0; i < K; ++i) {
        const int n = 2 * i;
        const double tPn = ((n + 1) * I(n + 1) + (n > 0 ? n * I(n - 1) : 0.0)) / (2.0 * n + 1.0);
        s += t.coef[i] * std::sqrt(n + 0.5) * tPn;
    }
    return s;
}

void gl_nodes(int n, std::vector<double> &x, std::vector<double> &w)
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

}  // namespace

void build_tables_pow2(Tables *t)
{
    const Params &prm = t->prm;
    const double c1 = phi2_raw(*t, 1.0);
    auto phi2 = [&](double x) { return x >= 1.0 ? 1.0 : phi2_raw(*t, x) / c1; };
    // ---- g2(tt) = Phi2(sqrt tt)/tt, Chebyshev series in 2 tt - 1
    const int M = 48;
    std::vector<double> cf(M);
    {
        std::vector<double> f(M);
        for (int k = 0; k < M; ++k) {
            const double tt = 0.5 * (std::cos(M_PI * (k + 0.5) / M) + 1.0);
            f[k] = phi2(std::sqrt(tt)) / tt;
        }
        for (int j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int k = 0; k < M; ++k) acc += f[k] * std::cos(M_PI * j * (k + 0.5) / M);
            cf[j] = (j == 0 ? 1.0 : 2.0) * acc / M;
        }
    }
    auto g2 = [&](double tt) {
        const double u = 2.0 * tt - 1.0;
        double b1 = 0.0, b2 = 0.0;
        for (int k = M - 1; k >= 1; --k) {
            const double b0 = cf[k] + 2.0 * u * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
        return cf[0] + u * b1 - b2;
    };
    {
        int deg = M - 1;
        while (deg > 0 && std::fabs(cf[deg]) < 1e-14 * std::fabs(cf[0])) deg--;
        t->gdeg = deg;
        t->gcheb.assign(cf.begin(), cf.begin() + deg + 1);
        int deg32 = deg;
        while (deg32 > 0 && std::fabs(cf[deg32]) < 1e-7 * std::fabs(cf[0])) deg32--;
        t->gdeg32 = deg32;
    }
    std::vector<double> gx, gw;
    gl_nodes(20, gx, gw);
    // radial transform (4 pi/k) int_a^b f(r) r sin(kr) dr on npan panels
    auto radial = [&](auto f, double a, double b, int npan, double k) {
        double acc = 0.0;
        for (int q = 0; q < npan; ++q) {
            const double lo = a + (b - a) * q / npan, hi = a + (b - a) * (q + 1) / npan;
            for (size_t i = 0; i < gx.size(); ++i) {
                const double r = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[i];
                acc += 0.5 * (hi - lo) * gw[i] * f(r) * r * (k == 0.0 ? r : std::sin(k * r) / k);
            }
        }
        return 4.0 * M_PI * acc;
    };
    // ---- level-0 difference-kernel weights, layout [m1][m3][m2]
    {
        auto d0 = [&](double r) { return (r < 0.5) ? 4.0 * g2(4.0 * r * r) - g2(r * r) : 1.0 / (r * r) - g2(r * r); };
        const double h = 2.0 * M_PI / 3.0, fac = std::pow(h / (2.0 * M_PI), 3);
        const int nf = prm.nf, maxk2 = 3 * nf * nf;
        std::vector<double> memo(maxk2 + 1);
        for (int k2 = 0; k2 <= maxk2; ++k2) {
            const double k = h * std::sqrt((double)k2);
            memo[k2] = fac * (radial(d0, 0.0, 0.5, 16, k) + radial(d0, 0.5, 1.0, 16, k));
        }
        t->wd0.assign((size_t)t->nh * t->nn * t->nn, 0.0);
        for (int m1 = -nf; m1 <= nf; ++m1)
            for (int m3 = 0; m3 <= nf; ++m3)
                for (int m2 = -nf; m2 <= nf; ++m2)
                    t->wd0[((size_t)(m1 + nf) * t->nh + m3) * t->nn + (m2 + nf)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
    // ---- root window weights (hw/2pi)^3 What_0(hw |m|), layout [m3][m2][m1]
    {
        const double a = std::sqrt(3.0);
        auto w0 = [&](double r) {
            const double m0 = (r < 1.0) ? g2(r * r) : 1.0 / (r * r);
            if (r <= a) return m0;
            if (r >= a + 2.0) return 0.0;
            const double y = r - a - 1.0;
            return m0 * 0.5 * (1.0 - (y >= 0.0 ? 1.0 : -1.0) * phi_window(*t, std::fabs(y)));
        };
        const double h = prm.hw, fac = std::pow(h / (2.0 * M_PI), 3);
        const int nw = prm.nw, maxk2 = 3 * nw * nw;
        std::vector<double> memo(maxk2 + 1);
        for (int k2 = 0; k2 <= maxk2; ++k2) {
            const double k = h * std::sqrt((double)k2);
            memo[k2] = fac * (radial(w0, 0.0, 1.0, 20, k) + radial(w0, 1.0, a, 10, k) + radial(w0, a, a + 2.0, 20, k));
        }
        t->ww.assign((size_t)t->nwh * t->nwn * t->nwn, 0.0);
        for (int m3 = 0; m3 <= nw; ++m3)
            for (int m2 = -nw; m2 <= nw; ++m2)
                for (int m1 = -nw; m1 <= nw; ++m1)
                    t->ww[((size_t)m3 * t->nwn + (m2 + nw)) * t->nwn + (m1 + nw)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
}

// ------------------------------------------------------ parameter search
// For a tolerance without a row in the parameter table (Sec. 3.7): c from
// the rule c ~ log(1/eps) of eq. pswfcvalue (or the caller's c), then the
// smallest plane-wave half width n_f and the smallest proxy order p that
// each meet eps, both measured on the level-0 difference kernel
// D_0(r) = (Phi(2r) - Phi(r))/r (box side 1) relative to D_0(0) = psi(0)/c_0:
//  * n_f: the trapezoidal sum over the modes m in [-n_f, n_f]^3 at spacing
//    h = 2 pi/3 against D_0(|x|) for offsets x in the colleague range
//    [-2, 2]^3;
//  * p: the tensor interpolant on p first-kind Chebyshev nodes per axis of
//    y -> D_0(|x - y|) over the source box [-1/2, 1/2]^3 against D_0 itself,
//    for targets x in [-3/2, 3/2]^3 (the box and its colleagues).
// Sample points are a fixed Halton sequence, so the search is deterministic.
// At the table's tolerances (with its c) it returns the table's N_1 and p.
namespace {

double halton(int i, int base)
{
    double f = 1.0, r = 0.0;
    for (int k = i + 1; k > 0; k /= base) {
        f /= base;
        r += f * (k % base);
    }
    return r;
}

struct D0Eval {
    const Tables &t;
    double d00;
    explicit D0Eval(const Tables &tt) : t(tt), d00(tt.psi0 / tt.c0) {}
    // g(t) = Phi(sqrt t)/sqrt t on [0, 1] from its Chebyshev series in 2t - 1
    double g(double tt) const
    {
        const double u = 2.0 * tt - 1.0;
        double b1 = 0.0, b2 = 0.0;
        for (int k = t.gdeg; k >= 1; --k) {
            const double b0 = t.gcheb[k] + 2.0 * u * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
        return t.gcheb[0] + u * b1 - b2;
    }
    // D_0(r) = (Phi(2r) - Phi(r))/r, Phi(x) = x g(x^2) below 1 and 1 beyond
    double operator()(double r) const
    {
        if (r >= 1.0) return 0.0;
        const double inner = g(r * r);
        if (2.0 * r < 1.0) return 2.0 * g(4.0 * r * r) - inner;
        return 1.0 / r - inner;
    }
};

double pw_error(const Tables &t, const D0Eval &D0, int nf)
{
    const double c = t.prm.c, h = 2.0 * M_PI / 3.0;
    const int nn = 2 * nf + 1, maxk2 = 3 * nf * nf;
    std::vector<double> w(maxk2 + 1);
    // weights (h/2pi)^3 Dhat_0(h|m|) of the 1/r split,
    // Dhat_0(k) = 4 pi [psi(k/(2c)) - psi(k/c)]/(psi(0) k^2), Dhat_0(0) = 2 pi (c_2/c_0)(1 - 1/4)
    const double fac = std::pow(h / (2.0 * M_PI), 3);
    w[0] = fac * 2.0 * M_PI * t.c2 / t.c0 * (1.0 - 0.25);
    for (int k2 = 1; k2 <= maxk2; ++k2) {
        double k = h * std::sqrt((double)k2);
        w[k2] = fac * 4.0 * M_PI * (pswf_eval(t, 0.5 * k / c) - pswf_eval(t, k / c)) / (t.psi0 * k * k);
    }
    std::vector<double> er(3 * nn), ei(3 * nn);
    double err = 0.0;
    const int NS = 96;
    for (int s = 0; s < NS + 24; ++s) {
        double x[3];
        if (s < NS) {
            for (int d = 0; d < 3; ++d) x[d] = 4.0 * halton(s, d == 0 ? 2 : (d == 1 ? 3 : 5)) - 2.0;
        } else {  // points on an axis and on the diagonal
            double u = 2.0 * ((s - NS) % 12) / 11.0;
            x[0] = u;
            x[1] = x[2] = (s - NS < 12) ? 0.0 : u;
        }
        for (int d = 0; d < 3; ++d)
            for (int m = -nf; m <= nf; ++m) {
                er[d * nn + m + nf] = std::cos(h * m * x[d]);
                ei[d * nn + m + nf] = std::sin(h * m * x[d]);
            }
        double sum = 0.0;
        for (int m1 = -nf; m1 <= nf; ++m1)
            for (int m2 = -nf; m2 <= nf; ++m2) {
                const double ar = er[m1 + nf] * er[nn + m2 + nf] - ei[m1 + nf] * ei[nn + m2 + nf];
                const double ai = er[m1 + nf] * ei[nn + m2 + nf] + ei[m1 + nf] * er[nn + m2 + nf];
                const int b2 = m1 * m1 + m2 * m2;
                for (int m3 = -nf; m3 <= nf; ++m3)
                    sum += w[b2 + m3 * m3] * (ar * er[2 * nn + m3 + nf] - ai * ei[2 * nn + m3 + nf]);
            }
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        err = std::max(err, std::fabs(sum - D0(r)));
    }
    return err / D0.d00;
}

double proxy_error(const Tables &t, const D0Eval &D0, int p)
{
    std::vector<double> nodes(p), bw(p);
    for (int j = 0; j < p; ++j) {
        nodes[j] = 0.5 * std::cos(M_PI * (j + 0.5) / p);
        bw[j] = ((j & 1) ? -1.0 : 1.0) * std::sin((2 * j + 1) * M_PI / (2.0 * p));
    }
    auto basis = [&](double y, double *out) {
        for (int a = 0; a < p; ++a)
            if (y == nodes[a]) {
                for (int b = 0; b < p; ++b) out[b] = (a == b) ? 1.0 : 0.0;
                return;
            }
        double den = 0.0;
        for (int a = 0; a < p; ++a) den += (out[a] = bw[a] / (y - nodes[a]));
        for (int a = 0; a < p; ++a) out[a] /= den;
    };
    const int NX = 48, NY = 64;
    std::vector<double> V((size_t)p * p * p), L((size_t)3 * NY * p), ys((size_t)3 * NY), t1((size_t)p * p), t2(p);
    for (int j = 0; j < NY; ++j)
        for (int d = 0; d < 3; ++d) {
            ys[3 * j + d] = halton(j + 7, d == 0 ? 7 : (d == 1 ? 11 : 13)) - 0.5;
            basis(ys[3 * j + d], &L[((size_t)d * NY + j) * p]);
        }
    double err = 0.0;
    for (int s = 0; s < NX; ++s) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = 3.0 * halton(s + 3, d == 0 ? 2 : (d == 1 ? 3 : 5)) - 1.5;
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j)
                for (int k = 0; k < p; ++k) {
                    const double a = x[0] - nodes[i], b = x[1] - nodes[j], cc = x[2] - nodes[k];
                    V[((size_t)i * p + j) * p + k] = D0(std::sqrt(a * a + b * b + cc * cc));
                }
        for (int yj = 0; yj < NY; ++yj) {
            const double *l1 = &L[(size_t)yj * p], *l2 = &L[((size_t)NY + yj) * p], *l3 = &L[((size_t)2 * NY + yj) * p];
            double v = 0.0;
            for (int i = 0; i < p; ++i) {
                double si = 0.0;
                for (int j = 0; j < p; ++j) {
                    const double *row = &V[((size_t)i * p + j) * p];
                    double sj = 0.0;
                    for (int k = 0; k < p; ++k) sj += l3[k] * row[k];
                    si += l2[j] * sj;
                }
                v += l1[i] * si;
            }
            const double a = x[0] - ys[3 * yj], b = x[1] - ys[3 * yj + 1], cc = x[2] - ys[3 * yj + 2];
            err = std::max(err, std::fabs(v - D0(std::sqrt(a * a + b * b + cc * cc))));
        }
    }
    return err / D0.d00;
}

}  // namespace

void search_params(double tol, double c, Params *out, double *err_nf, double *err_p)
{
    Params prm{};
    prm.tol = tol;
    prm.c = c;
    prm.nf = 1;
    prm.p = 2;
    prm.nw = 1;
    prm.hw = 1.0;
    Tables t;
    build_tables(prm, &t, 3);
    const D0Eval D0(t);
    // errors fall with n_f and p until the split's own floor; start below
    // the table's ratios (n_f ~ 0.87 c / (pi 2/3) ... p ~ 1.3 c) and step up
    int nf = std::max(1, (int)std::floor(0.5 * c)), p = std::max(2, (int)std::floor(0.9 * c));
    double e = pw_error(t, D0, nf);
    while (nf > 1 && e <= tol) e = pw_error(t, D0, --nf);  // make sure the start is below the answer
    while (e > tol && nf < 64) e = pw_error(t, D0, ++nf);
    if (err_nf) *err_nf = e;
    double ep = proxy_error(t, D0, p);
    while (p > 2 && ep <= tol) ep = proxy_error(t, D0, --p);
    while (ep > tol && p < 64) ep = proxy_error(t, D0, ++p);
    if (err_p) *err_p = ep;
    out->tol = tol;
    out->c = c;
    out->nf = nf;
    out->p = p;
}

}  // namespace dmk
