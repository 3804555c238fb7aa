/*
 * dmk.c -- Steps 1-5 of the discrete DMK algorithm (Sec. 3.5, "The full DMK
 * algorithm for discrete sources") for the 3-D Laplace kernel with the PSWF
 * split of Sec. 3.7, plus direct summation.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain FP64 loops; the
 * tensor-product operators are applied one dimension at a time (separation
 * of variables), as the paper prescribes for every transform.
 *
 * Conventions fixed here where the paper leaves room (each is also listed
 * with its reason in the design notes of the repository):
 *  - box side s_l = 2^{-l}, root box [-1/2,1/2]^3;
 *  - plane-wave spacing h_l = 2 pi / (3 s_l): D_l vanishes beyond s_l and
 *    colleague offsets reach 2 s_l per axis, so the period 2 pi/h_l = 3 s_l
 *    keeps periodic images out of range (eq. fourierspacing, with the support
 *    of the PSWF difference kernel);
 *  - trapezoidal weights w_{l,m} = (h_l/2pi)^3 Dhat_l(h_l |m|) (eq. wlmdef
 *    with the rectangle-rule factor h^3);
 *  - W_0 (root only) uses the truncated-kernel window with A = (1+sqrt 3) s_0
 *    and transform prefactor 8 pi;
 *  - D_l is applied at level l for l = 0 .. L_s - 1, where L_s is the level of
 *    a source's terminal box; the root applies W_0 and D_0;
 *  - every non-leaf box hands its local expansion down to its children;
 *  - residual lists are source-centric: a terminal box T at level l acts on
 *    all targets in the subtrees of its colleagues and, if T is a leaf, in
 *    its coarse-neighbour leaves (Step 4, eq. nearpotential remark);
 *  - pairs at distance exactly zero (the self pair included) contribute
 *    -M_l(0) q_j, which removes the smooth part the far field carried
 *    (Step 5 self-interaction correction, eq. laplacesum2self).
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

/* threads of the following parallel regions (n >= 1); returns the previous count */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    const int prev = omp_get_max_threads();
    if (n >= 1) omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#include "cheb.h"

void cheb_T(int p, double x, double *T)
{
    T[0] = 1.0;
    if (p > 1) T[1] = x;
    for (int n = 2; n < p; ++n) T[n] = 2.0 * x * T[n - 1] - T[n - 2];
}

/* row of the interpolation matrix U = E V^{-1} at one point */
void cheb_interp_row(const cheb_t *ch, double xi, double *u)
{
    int p = ch->p;
    double T[64];
    cheb_T(p, xi, T);
    for (int a = 0; a < p; ++a) {
        double s = 0.0;
        for (int n = 0; n < p; ++n) s += T[n] * ch->vinv[n * p + a];
        u[a] = s;
    }
}

void cheb_init(int p, cheb_t *ch)
{
    ch->p = p;
    ch->x = (double *)malloc((size_t)p * sizeof(double));
    for (int i = 0; i < p; ++i) ch->x[i] = cos(M_PI * (i + 0.5) / p);
    /* Gauss-Jordan inverse of V with partial pivoting */
    double *M = (double *)malloc((size_t)p * 2 * p * sizeof(double));
    double T[64];
    for (int i = 0; i < p; ++i) {
        cheb_T(p, ch->x[i], T);
        for (int j = 0; j < p; ++j) {
            M[i * 2 * p + j] = T[j];
            M[i * 2 * p + p + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < p; ++col) {
        int piv = col;
        for (int r = col + 1; r < p; ++r)
            if (fabs(M[r * 2 * p + col]) > fabs(M[piv * 2 * p + col])) piv = r;
        if (piv != col)
            for (int j = 0; j < 2 * p; ++j) {
                double tmp = M[col * 2 * p + j];
                M[col * 2 * p + j] = M[piv * 2 * p + j];
                M[piv * 2 * p + j] = tmp;
            }
        double d = M[col * 2 * p + col];
        for (int j = 0; j < 2 * p; ++j) M[col * 2 * p + j] /= d;
        for (int r = 0; r < p; ++r) {
            if (r == col) continue;
            double f = M[r * 2 * p + col];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * p; ++j) M[r * 2 * p + j] -= f * M[col * 2 * p + j];
        }
    }
    ch->vinv = (double *)malloc((size_t)p * p * sizeof(double));
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) ch->vinv[i * p + j] = M[i * 2 * p + p + j];
    free(M);
    for (int s = 0; s < 2; ++s) {
        double sigma = s ? 1.0 : -1.0;
        ch->A[s] = (double *)malloc((size_t)p * p * sizeof(double));
        double u[64];
        for (int i = 0; i < p; ++i) {
            cheb_interp_row(ch, 0.5 * (ch->x[i] + sigma), u);
            for (int a = 0; a < p; ++a) ch->A[s][a * p + i] = u[a];
        }
    }
}

void cheb_free(cheb_t *ch)
{
    free(ch->x); free(ch->vinv); free(ch->A[0]); free(ch->A[1]);
}

/* --------------------------------------------------- tensor mode products
 * T is a dense 3-index array t[i0][i1][i2] with dims n[0..2].  A mode-k
 * product with an (mo x n[k]) matrix M replaces axis k by mo entries. */
static void mode_real(const double *in, const int n[3], int k, const double *M, int mo,
                      double *out)
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

static void mode_cplx(const cplx *in, const int n[3], int k, const cplx *M, int mo, cplx *out)
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

/* proxies rho[p^3] -> outgoing plane waves Phi[(2nm+1)^3]
 * Phi_m = sum_j exp(-i h m.(r_j - c)) rho_j,  r_j - c = (s/2) x_j  (eq. outgoingexpansion2) */
static void proxy_to_pw(const cheb_t *ch, const double *rho, double h, double s, int nm, cplx *phi)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *E = (cplx *)malloc((size_t)n * p * sizeof(cplx));
    for (int m = 0; m < n; ++m)
        for (int j = 0; j < p; ++j) E[m * p + j] = cexp(-I * h * (m - nm) * 0.5 * s * ch->x[j]);
    cplx *t0 = (cplx *)malloc((size_t)p * p * p * sizeof(cplx));
    for (int i = 0; i < p * p * p; ++i) t0[i] = rho[i];
    int d0[3] = {p, p, p};
    cplx *t1 = (cplx *)malloc((size_t)p * p * n * sizeof(cplx));
    mode_cplx(t0, d0, 2, E, n, t1);
    int d1[3] = {p, p, n};
    cplx *t2 = (cplx *)malloc((size_t)p * n * n * sizeof(cplx));
    mode_cplx(t1, d1, 1, E, n, t2);
    int d2[3] = {p, n, n};
    mode_cplx(t2, d2, 0, E, n, phi);
    free(E); free(t0); free(t1); free(t2);
}

/* incoming plane waves Psi -> values on the box's Chebyshev grid
 * v_j += Re sum_m exp(+i h m.(r_j - c)) Psi_m  (eq. incomingexpansion2) */
static void pw_to_grid(const cheb_t *ch, const cplx *psi, double h, double s, int nm, double *v)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *G = (cplx *)malloc((size_t)p * n * sizeof(cplx));
    for (int j = 0; j < p; ++j)
        for (int m = 0; m < n; ++m) G[j * n + m] = cexp(I * h * (m - nm) * 0.5 * s * ch->x[j]);
    int d0[3] = {n, n, n};
    cplx *t1 = (cplx *)malloc((size_t)n * n * p * sizeof(cplx));
    mode_cplx(psi, d0, 2, G, p, t1);
    int d1[3] = {n, n, p};
    cplx *t2 = (cplx *)malloc((size_t)n * p * p * sizeof(cplx));
    mode_cplx(t1, d1, 1, G, p, t2);
    int d2[3] = {n, p, p};
    cplx *t3 = (cplx *)malloc((size_t)p * p * p * sizeof(cplx));
    mode_cplx(t2, d2, 0, G, p, t3);
    for (int i = 0; i < p * p * p; ++i) v[i] += creal(t3[i]);
    free(G); free(t1); free(t2); free(t3);
}

static void box_center(const orc_tree *t, int64_t b, double c[3])
{
    int l = t->level[b];
    uint64_t P = t->bkey[b];
    double s = ldexp(1.0, -l);
    for (int d = 0; d < 3; ++d) {
        uint64_t cd = 0;
        for (int bb = 0; bb < l; ++bb) cd |= ((P >> (3 * bb + (2 - d))) & 1ull) << bb;
        c[d] = -0.5 + ((double)cd + 0.5) * s;
    }
}

/* child position bits (x, y, z) of a box within its parent */
static void child_bits(const orc_tree *t, int64_t b, int o[3])
{
    uint64_t P = t->bkey[b];
    o[0] = (int)((P >> 2) & 1);
    o[1] = (int)((P >> 1) & 1);
    o[2] = (int)(P & 1);
}

int orc_dmk_eval(const orc_tree *t, const orc_params *pr, const orc_pswf *ps,
                 const double *charges, int keep, orc_dmk_result *res)
{
    return orc_dmk_eval_k(t, pr, ps, ORC_LAP3, 0.0, charges, keep, res);
}

int orc_dmk_eval_k(const orc_tree *t, const orc_params *pr, const orc_pswf *ps, int kern, double lam_in,
                   const double *charges, int keep, orc_dmk_result *res)
{
    memset(res, 0, sizeof(*res));
    if (t->dim != 3) return -1;
    const double lam = lam_in * t->side; /* Yukawa parameter in root-box units */
    if (kern == ORC_YUK3 && !(lam >= 1e-3)) return -1;
    if (kern != ORC_LAP3 && kern != ORC_YUK3 && kern != ORC_POW3) return -1;
    orc_pow2 p2;
    if (kern == ORC_POW3) orc_p2_init(ps, &p2);
    const int64_t n = t->n;
    const int p = pr->p, p3 = p * p * p;
    const int nf = pr->nf, nn = 2 * nf + 1, n3 = nn * nn * nn;
    const int nw = pr->nw, nwn = 2 * nw + 1, nw3 = nwn * nwn * nwn;
    const int64_t nbox = t->nbox;
    res->n = n;
    res->p = p;
    res->nf = nf;
    res->u = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    res->ufar = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    res->ures = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    if (n == 0) return 0;

    double *q = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) q[i] = charges[t->perm[i]];

    cheb_t ch;
    cheb_init(p, &ch);
    double **proxy = (double **)calloc((size_t)nbox, sizeof(double *));
    double **local = (double **)calloc((size_t)nbox, sizeof(double *));

    /* ---- Step 2: upward pass.  Leaves: proxy charges from sources
       (Def. 2.1, eq. proxynd); parents: merge children with T_c2p (Lemma 2.1). */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nbox; ++b) {
        if (!t->leaf[b] || t->pcount[b] == 0) continue;
        double c[3], s = ldexp(1.0, -t->level[b]);
        box_center(t, b, c);
        double *rho = (double *)calloc((size_t)p3, sizeof(double));
        double u0[64], u1[64], u2[64];
        for (int64_t i = t->pstart[b]; i < t->pstart[b] + t->pcount[b]; ++i) {
            const double *x = &t->xs[3 * i];
            cheb_interp_row(&ch, 2.0 * (x[0] - c[0]) / s, u0);
            cheb_interp_row(&ch, 2.0 * (x[1] - c[1]) / s, u1);
            cheb_interp_row(&ch, 2.0 * (x[2] - c[2]) / s, u2);
            for (int a = 0; a < p; ++a)
                for (int bb = 0; bb < p; ++bb)
                    for (int cc = 0; cc < p; ++cc)
                        rho[(a * p + bb) * p + cc] += u0[a] * u1[bb] * u2[cc] * q[i];
        }
        proxy[b] = rho;
    }
    for (int l = t->nlevels - 2; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = t->level_start[l]; b < t->level_start[l + 1]; ++b) {
            if (t->leaf[b] || t->pcount[b] == 0) continue;
            double *rho = (double *)calloc((size_t)p3, sizeof(double));
            double *tA = (double *)malloc((size_t)p3 * sizeof(double));
            double *tB = (double *)malloc((size_t)p3 * sizeof(double));
            int dims[3] = {p, p, p};
            for (int k = 0; k < 8; ++k) {
                int64_t cb = t->child0[b] + k;
                if (!proxy[cb]) continue;
                int o[3];
                child_bits(t, cb, o);
                mode_real(proxy[cb], dims, 2, ch.A[o[2]], p, tA);
                mode_real(tA, dims, 1, ch.A[o[1]], p, tB);
                mode_real(tB, dims, 0, ch.A[o[0]], p, tA);
                for (int i = 0; i < p3; ++i) rho[i] += tA[i];
            }
            free(tA); free(tB);
            proxy[b] = rho;
            if (!keep)
                for (int k = 0; k < 8; ++k) {
                    int64_t cb = t->child0[b] + k;
                    if (!t->fout[cb]) { free(proxy[cb]); proxy[cb] = NULL; }
                }
        }
    }

    /* plane-wave weights, memoised by |m|^2 */
    const double hw = pr->hw;
    double *wW = (double *)malloc((size_t)nw3 * sizeof(double));
    {
        double fac = pow(hw / (2.0 * M_PI), 3);
        int maxk2 = 3 * nw * nw;
        double *memo = (double *)malloc((size_t)(maxk2 + 1) * sizeof(double));
        for (int k2 = 0; k2 <= maxk2; ++k2) {
            const double k = hw * sqrt((double)k2);
            memo[k2] = fac * (kern == ORC_YUK3   ? orc_y3_w0hat(ps, lam, k)
                              : kern == ORC_POW3 ? orc_p2_w0hat(&p2, k)
                                                 : orc_w0hat(ps, k));
        }
        for (int a = 0; a < nwn; ++a)
            for (int bb = 0; bb < nwn; ++bb)
                for (int cc = 0; cc < nwn; ++cc) {
                    int k2 = (a - nw) * (a - nw) + (bb - nw) * (bb - nw) + (cc - nw) * (cc - nw);
                    wW[(a * nwn + bb) * nwn + cc] = memo[k2];
                }
        free(memo);
    }
    int maxk2 = 3 * nf * nf;
    double *dmemo = (double *)malloc((size_t)(maxk2 + 1) * sizeof(double));

    /* ---- root: windowed kernel W_0 over the whole unit box */
    {
        int64_t r = 0;
        cplx *phi = (cplx *)malloc((size_t)nw3 * sizeof(cplx));
        proxy_to_pw(&ch, proxy[r], hw, 1.0, nw, phi);
        for (int i = 0; i < nw3; ++i) phi[i] *= wW[i];
        local[r] = (double *)calloc((size_t)p3, sizeof(double));
        pw_to_grid(&ch, phi, hw, 1.0, nw, local[r]);
        free(phi);
    }

    /* ---- Step 3: downward pass */
    cplx **phi = (cplx **)calloc((size_t)nbox, sizeof(cplx *));
    for (int l = 0; l < t->nlevels; ++l) {
        const int64_t b0 = t->level_start[l], b1 = t->level_start[l + 1];
        const double s = ldexp(1.0, -l);
        const double h = 2.0 * M_PI / (3.0 * s);
        double fac = pow(h / (2.0 * M_PI), 3);
        for (int k2 = 0; k2 <= maxk2; ++k2) {
            const double k = h * sqrt((double)k2);
            dmemo[k2] = fac * (kern == ORC_YUK3   ? orc_y3_dhat(ps, lam, l, k)
                               : kern == ORC_POW3 ? orc_p2_dhat(&p2, l, k)
                                                  : orc_dhat(ps, l, k));
        }

        /* outgoing expansions Phi_l(B) for F_out boxes */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->fout[b]) continue;
            phi[b] = (cplx *)malloc((size_t)n3 * sizeof(cplx));
            proxy_to_pw(&ch, proxy[b], h, s, nf, phi[b]);
        }
        /* incoming expansions by diagonal translation (eq. diagonaltranslation),
           then local values on the Chebyshev grid (eq. incomingexpansion2) */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->fin[b] || t->pcount[b] == 0) continue;
            double cb[3];
            box_center(t, b, cb);
            cplx *psi = (cplx *)calloc((size_t)n3, sizeof(cplx));
            cplx e0[64], e1[64], e2[64];
            for (int k = 0; k < 27; ++k) {
                int64_t sb = t->colleague[b * 27 + k];
                if (sb < 0 || !t->fout[sb]) continue;
                double cs[3];
                box_center(t, sb, cs);
                for (int m = 0; m < nn; ++m) {
                    e0[m] = cexp(I * h * (m - nf) * (cb[0] - cs[0]));
                    e1[m] = cexp(I * h * (m - nf) * (cb[1] - cs[1]));
                    e2[m] = cexp(I * h * (m - nf) * (cb[2] - cs[2]));
                }
                for (int a = 0; a < nn; ++a)
                    for (int bb = 0; bb < nn; ++bb)
                        for (int cc = 0; cc < nn; ++cc) {
                            int idx = (a * nn + bb) * nn + cc;
                            psi[idx] += e0[a] * e1[bb] * e2[cc] * phi[sb][idx];
                        }
            }
            for (int a = 0; a < nn; ++a)
                for (int bb = 0; bb < nn; ++bb)
                    for (int cc = 0; cc < nn; ++cc) {
                        int k2 = (a - nf) * (a - nf) + (bb - nf) * (bb - nf) + (cc - nf) * (cc - nf);
                        psi[(a * nn + bb) * nn + cc] *= dmemo[k2];
                    }
            if (!local[b]) local[b] = (double *)calloc((size_t)p3, sizeof(double));
            pw_to_grid(&ch, psi, h, s, nf, local[b]);
            free(psi);
        }
        /* leaves: evaluate the far potential at their targets */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->leaf[b] || t->pcount[b] == 0) continue;
            double c[3];
            box_center(t, b, c);
            double u0[64], u1[64], u2[64];
            for (int64_t i = t->pstart[b]; i < t->pstart[b] + t->pcount[b]; ++i) {
                const double *x = &t->xs[3 * i];
                cheb_interp_row(&ch, 2.0 * (x[0] - c[0]) / s, u0);
                cheb_interp_row(&ch, 2.0 * (x[1] - c[1]) / s, u1);
                cheb_interp_row(&ch, 2.0 * (x[2] - c[2]) / s, u2);
                double acc = 0.0;
                for (int a = 0; a < p; ++a)
                    for (int bb = 0; bb < p; ++bb)
                        for (int cc = 0; cc < p; ++cc)
                            acc += local[b][(a * p + bb) * p + cc] * u0[a] * u1[bb] * u2[cc];
                res->ufar[i] = acc;
            }
        }
        /* split local expansions to children (Lemma 2.2) */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (t->leaf[b] || t->pcount[b] == 0) continue;
            double *tA = (double *)malloc((size_t)p3 * sizeof(double));
            double *tB = (double *)malloc((size_t)p3 * sizeof(double));
            double *AT[2] = {(double *)malloc((size_t)p * p * sizeof(double)),
                             (double *)malloc((size_t)p * p * sizeof(double))};
            for (int sgn = 0; sgn < 2; ++sgn)
                for (int i = 0; i < p; ++i)
                    for (int a = 0; a < p; ++a) AT[sgn][i * p + a] = ch.A[sgn][a * p + i];
            int dims[3] = {p, p, p};
            for (int k = 0; k < 8; ++k) {
                int64_t cbx = t->child0[b] + k;
                if (t->pcount[cbx] == 0) continue;
                int o[3];
                child_bits(t, cbx, o);
                mode_real(local[b], dims, 2, AT[o[2]], p, tA);
                mode_real(tA, dims, 1, AT[o[1]], p, tB);
                mode_real(tB, dims, 0, AT[o[0]], p, tA);
                local[cbx] = (double *)malloc((size_t)p3 * sizeof(double));
                memcpy(local[cbx], tA, (size_t)p3 * sizeof(double));
            }
            free(tA); free(tB); free(AT[0]); free(AT[1]);
        }
        for (int64_t b = b0; b < b1; ++b) {
            free(phi[b]);
            phi[b] = NULL;
            if (!keep) {
                free(local[b]); local[b] = NULL;
                free(proxy[b]); proxy[b] = NULL;
            }
        }
    }
    free(phi);
    free(wW);
    free(dmemo);

    /* ---- Steps 4-5: residual sums and self-interaction correction */
    orc_split3 sp3;
    memset(&sp3, 0, sizeof(sp3));
    if (kern == ORC_YUK3) orc_y3_split_init(ps, lam, t->nlevels, &sp3);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t T = 0; T < nbox; ++T) {
        if (!t->terminal[T] || t->pcount[T] == 0) continue;
        const int l = t->level[T];
        const double s = ldexp(1.0, -l);
        const double m0 = (kern == ORC_YUK3) ? sp3.self[l] : (kern == ORC_POW3) ? orc_p2_m0(&p2, l) : orc_split_m0(ps, l);
        int64_t lists[27 + 7][2];
        int nl = 0;
        for (int k = 0; k < 27; ++k) {
            int64_t cb = t->colleague[T * 27 + k];
            if (cb < 0 || t->pcount[cb] == 0) continue;
            lists[nl][0] = t->pstart[cb];
            lists[nl][1] = t->pstart[cb] + t->pcount[cb];
            nl++;
        }
        if (t->leaf[T])
            for (int k = 0; k < t->ncoarse[T]; ++k) {
                int64_t cb = t->coarse[T * 7 + k];
                if (t->pcount[cb] == 0) continue;
                lists[nl][0] = t->pstart[cb];
                lists[nl][1] = t->pstart[cb] + t->pcount[cb];
                nl++;
            }
        for (int64_t j = t->pstart[T]; j < t->pstart[T] + t->pcount[T]; ++j) {
            const double *y = &t->xs[3 * j];
            for (int li = 0; li < nl; ++li)
                for (int64_t i = lists[li][0]; i < lists[li][1]; ++i) {
                    const double *x = &t->xs[3 * i];
                    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    double contrib;
                    if (r == 0.0) contrib = -m0 * q[j];
                    else if (r < s)
                        contrib = (kern == ORC_YUK3   ? orc_y3_residual(&sp3, l, r)
                                   : kern == ORC_POW3 ? orc_p2_r(&p2, l, r)
                                                      : orc_split_r(ps, l, r)) *
                                  q[j];
                    else continue;
#pragma omp atomic
                    res->ures[i] += contrib;
                }
        }
    }

    if (kern == ORC_YUK3) orc_y3_split_free(&sp3);
    /* unit change: 1/(4 pi S) for the 1/r kernels, 1/S^2 for 1/r^2 */
    const double scale = (kern == ORC_POW3) ? 1.0 / (t->side * t->side) : 1.0 / (4.0 * M_PI * t->side);
    for (int64_t i = 0; i < n; ++i) res->u[t->perm[i]] = (res->ufar[i] + res->ures[i]) * scale;

    if (keep) {
        res->proxy = proxy;
        res->local = local;
    } else {
        for (int64_t b = 0; b < nbox; ++b) { free(proxy[b]); free(local[b]); }
        free(proxy);
        free(local);
    }
    cheb_free(&ch);
    free(q);
    return 0;
}

void orc_dmk_result_free(const orc_tree *t, orc_dmk_result *res)
{
    if (res->proxy) {
        for (int64_t b = 0; b < t->nbox; ++b) free(res->proxy[b]);
        free(res->proxy);
    }
    if (res->local) {
        for (int64_t b = 0; b < t->nbox; ++b) free(res->local[b]);
        free(res->local);
    }
    free(res->u); free(res->ufar); free(res->ures);
    memset(res, 0, sizeof(*res));
}

/* u_i = sum_{j != i, r_ij > 0} q_j / (4 pi r_ij)  (eq. laplacesum), Neumaier sum */
void orc_direct(int64_t n, const double *pts, const double *q, int64_t nt, const int64_t *tidx,
                double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tidx[t];
        double s = 0.0, comp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pts[3 * i] - pts[3 * j], dy = pts[3 * i + 1] - pts[3 * j + 1],
                   dz = pts[3 * i + 2] - pts[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            double v = q[j] / r, tsum = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - tsum) + v;
            else comp += (v - tsum) + s;
            s = tsum;
        }
        out[t] = (s + comp) / (4.0 * M_PI);
    }
}

#include <time.h>
static double wall(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

int orc_dmk_run(int64_t n, const double *pts, const double *q, double tol, int ns, int maxdepth,
                double *u, double *times)
{
    orc_params pr;
    if (orc_params_for(tol, &pr)) return -1;
    double t0 = wall();
    orc_pswf ps;
    orc_pswf_init(pr.c, &ps);
    orc_tree tr;
    if (orc_tree_build(3, n, pts, ns, maxdepth, &tr)) return -2;
    double t1 = wall();
    orc_dmk_result res;
    int rc = orc_dmk_eval(&tr, &pr, &ps, q, 0, &res);
    double t2 = wall();
    if (rc == 0) memcpy(u, res.u, (size_t)n * sizeof(double));
    orc_dmk_result_free(&tr, &res);
    orc_tree_free(&tr);
    if (times) { times[0] = t1 - t0; times[1] = t2 - t1; }
    return rc;
}
