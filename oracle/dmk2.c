/*
 * dmk2.c -- the discrete DMK algorithm (Sec. 3.5, Steps 1-5) in two
 * dimensions, for K(r) = -log(r)/(2 pi) and K(r) = K_0(lambda r) with the
 * Fourier-space PSWF split of Sec. 4.6 (see split2.c), plus direct summation.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain FP64 loops.
 *
 * The conventions of the 3-D driver carry over with d = 2: box side
 * s_l = 2^{-l}, root box [-1/2,1/2]^2, plane-wave spacing h_l = 2 pi/(3 s_l)
 * and weights (h_l/2pi)^2 Dhat_l(h_l |m|); the root carries the windowed
 * kernel W_0 (truncation radius (1 + sqrt 2) s_0) and D_0 with itself as
 * colleague; D_l acts at levels l < L_s, L_s the level of a source's terminal
 * box; every non-leaf box hands its local expansion to its children;
 * residual lists are source-centric (3x3 colleagues, coarse-neighbour leaves);
 * pairs at distance zero contribute -M_{L_s}(0) times the charge.
 *
 * Units: the problem is solved on the scaled points x' = (x - centre)/S.
 * K_0(lambda S r') = K_0(lambda' r') with lambda' = lambda S.  For the log
 * kernel -log(S r')/(2 pi) = -log(r')/(2 pi) + C, C = -log(S)/(2 pi); a
 * constant kernel is its own far field, so C times the total charge is added
 * to the far part and C to M_L(0) in the r = 0 correction.
 */
#include "cheb.h"
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

/* mode products on a 2-index array t[i0][i1] of dims n[0..1] */
static void mode_real2(const double *in, const int n[2], int k, const double *M, int mo, double *out)
{
    int no[2] = {n[0], n[1]};
    no[k] = mo;
    for (int a = 0; a < no[0]; ++a)
        for (int b = 0; b < no[1]; ++b) {
            int o[2] = {a, b};
            double s = 0.0;
            for (int j = 0; j < n[k]; ++j) {
                int ii[2] = {a, b};
                ii[k] = j;
                s += M[o[k] * n[k] + j] * in[ii[0] * n[1] + ii[1]];
            }
            out[a * no[1] + b] = s;
        }
}

static void mode_cplx2(const cplx *in, const int n[2], int k, const cplx *M, int mo, cplx *out)
{
    int no[2] = {n[0], n[1]};
    no[k] = mo;
    for (int a = 0; a < no[0]; ++a)
        for (int b = 0; b < no[1]; ++b) {
            int o[2] = {a, b};
            cplx s = 0.0;
            for (int j = 0; j < n[k]; ++j) {
                int ii[2] = {a, b};
                ii[k] = j;
                s += M[o[k] * n[k] + j] * in[ii[0] * n[1] + ii[1]];
            }
            out[a * no[1] + b] = s;
        }
}

/* Phi_m = sum_j exp(-i h m.(r_j - c)) rho_j, r_j - c = (s/2) x_j */
static void proxy_to_pw2(const cheb_t *ch, const double *rho, double h, double s, int nm, cplx *phi)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *E = (cplx *)malloc((size_t)n * p * sizeof(cplx));
    for (int m = 0; m < n; ++m)
        for (int j = 0; j < p; ++j) E[m * p + j] = cexp(-I * h * (m - nm) * 0.5 * s * ch->x[j]);
    cplx *t0 = (cplx *)malloc((size_t)p * p * sizeof(cplx));
    for (int i = 0; i < p * p; ++i) t0[i] = rho[i];
    int d0[2] = {p, p};
    cplx *t1 = (cplx *)malloc((size_t)p * n * sizeof(cplx));
    mode_cplx2(t0, d0, 1, E, n, t1);
    int d1[2] = {p, n};
    mode_cplx2(t1, d1, 0, E, n, phi);
    free(E); free(t0); free(t1);
}

/* v_j += Re sum_m exp(+i h m.(r_j - c)) Psi_m */
static void pw_to_grid2(const cheb_t *ch, const cplx *psi, double h, double s, int nm, double *v)
{
    int p = ch->p, n = 2 * nm + 1;
    cplx *G = (cplx *)malloc((size_t)p * n * sizeof(cplx));
    for (int j = 0; j < p; ++j)
        for (int m = 0; m < n; ++m) G[j * n + m] = cexp(I * h * (m - nm) * 0.5 * s * ch->x[j]);
    int d0[2] = {n, n};
    cplx *t1 = (cplx *)malloc((size_t)n * p * sizeof(cplx));
    mode_cplx2(psi, d0, 1, G, p, t1);
    int d1[2] = {n, p};
    cplx *t2 = (cplx *)malloc((size_t)p * p * sizeof(cplx));
    mode_cplx2(t1, d1, 0, G, p, t2);
    for (int i = 0; i < p * p; ++i) v[i] += creal(t2[i]);
    free(G); free(t1); free(t2);
}

static void box_center2(const orc_tree *t, int64_t b, double c[2])
{
    int l = t->level[b];
    uint64_t P = t->bkey[b];
    double s = ldexp(1.0, -l);
    for (int d = 0; d < 2; ++d) {
        uint64_t cd = 0;
        for (int bb = 0; bb < l; ++bb) cd |= ((P >> (2 * bb + (1 - d))) & 1ull) << bb;
        c[d] = -0.5 + ((double)cd + 0.5) * s;
    }
}

static void child_bits2(const orc_tree *t, int64_t b, int o[2])
{
    uint64_t P = t->bkey[b];
    o[0] = (int)((P >> 1) & 1);
    o[1] = (int)(P & 1);
}

int orc_dmk2_eval(const orc_tree *t, const orc_params *pr, const orc_pswf *ps, int kern, double lam_in,
                  const double *charges, int keep, orc_dmk_result *res)
{
    memset(res, 0, sizeof(*res));
    if (t->dim != 2) return -1;
    const int64_t n = t->n;
    const int p = pr->p, p2 = p * p;
    const int nf = pr->nf, nn = 2 * nf + 1, n2 = nn * nn;
    const int nw = pr->nw, nwn = 2 * nw + 1, nw2 = nwn * nwn;
    const int64_t nbox = t->nbox;
    const double lam = (kern == ORC_YUK2) ? lam_in * t->side : 0.0;
    const double C = (kern == ORC_LOG2) ? -log(t->side) / (2.0 * M_PI) : 0.0;
    res->n = n;
    res->p = p;
    res->nf = nf;
    res->u = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    res->ufar = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    res->ures = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    if (n == 0) return 0;

    double *q = (double *)malloc((size_t)n * sizeof(double));
    double Q = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        q[i] = charges[t->perm[i]];
        Q += q[i];
    }
    orc_split2 sp;
    orc2_split_init(ps, kern, lam, t->nlevels, &sp);

    cheb_t ch;
    cheb_init(p, &ch);
    double **proxy = (double **)calloc((size_t)nbox, sizeof(double *));
    double **local = (double **)calloc((size_t)nbox, sizeof(double *));

    /* ---- Step 2: upward pass (Def. 2.1 for leaves, Lemma 2.1 for parents) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nbox; ++b) {
        if (!t->leaf[b] || t->pcount[b] == 0) continue;
        double c[2], s = ldexp(1.0, -t->level[b]);
        box_center2(t, b, c);
        double *rho = (double *)calloc((size_t)p2, sizeof(double));
        double u0[64], u1[64];
        for (int64_t i = t->pstart[b]; i < t->pstart[b] + t->pcount[b]; ++i) {
            const double *x = &t->xs[2 * i];
            cheb_interp_row(&ch, 2.0 * (x[0] - c[0]) / s, u0);
            cheb_interp_row(&ch, 2.0 * (x[1] - c[1]) / s, u1);
            for (int a = 0; a < p; ++a)
                for (int bb = 0; bb < p; ++bb) rho[a * p + bb] += u0[a] * u1[bb] * q[i];
        }
        proxy[b] = rho;
    }
    for (int l = t->nlevels - 2; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = t->level_start[l]; b < t->level_start[l + 1]; ++b) {
            if (t->leaf[b] || t->pcount[b] == 0) continue;
            double *rho = (double *)calloc((size_t)p2, sizeof(double));
            double *tA = (double *)malloc((size_t)p2 * sizeof(double));
            double *tB = (double *)malloc((size_t)p2 * sizeof(double));
            int dims[2] = {p, p};
            for (int k = 0; k < 4; ++k) {
                int64_t cb = t->child0[b] + k;
                if (!proxy[cb]) continue;
                int o[2];
                child_bits2(t, cb, o);
                mode_real2(proxy[cb], dims, 1, ch.A[o[1]], p, tA);
                mode_real2(tA, dims, 0, ch.A[o[0]], p, tB);
                for (int i = 0; i < p2; ++i) rho[i] += tB[i];
            }
            free(tA); free(tB);
            proxy[b] = rho;
            if (!keep)
                for (int k = 0; k < 4; ++k) {
                    int64_t cb = t->child0[b] + k;
                    if (!t->fout[cb]) { free(proxy[cb]); proxy[cb] = NULL; }
                }
        }
    }

    /* ---- root: windowed kernel W_0 over the whole unit box, plus the
       constant part of the log kernel */
    {
        const double hw = pr->hw, fac = pow(hw / (2.0 * M_PI), 2);
        cplx *phi = (cplx *)malloc((size_t)nw2 * sizeof(cplx));
        proxy_to_pw2(&ch, proxy[0], hw, 1.0, nw, phi);
        for (int a = 0; a < nwn; ++a)
            for (int bb = 0; bb < nwn; ++bb) {
                double k = hw * sqrt((double)((a - nw) * (a - nw) + (bb - nw) * (bb - nw)));
                phi[a * nwn + bb] *= fac * orc2_w0hat(ps, kern, lam, k);
            }
        local[0] = (double *)calloc((size_t)p2, sizeof(double));
        pw_to_grid2(&ch, phi, hw, 1.0, nw, local[0]);
        for (int i = 0; i < p2; ++i) local[0][i] += C * Q;
        free(phi);
    }

    /* ---- Step 3: downward pass */
    cplx **phi = (cplx **)calloc((size_t)nbox, sizeof(cplx *));
    const int maxk2 = 2 * nf * nf;
    double *dmemo = (double *)malloc((size_t)(maxk2 + 1) * sizeof(double));
    for (int l = 0; l < t->nlevels; ++l) {
        const int64_t b0 = t->level_start[l], b1 = t->level_start[l + 1];
        const double s = ldexp(1.0, -l);
        const double h = 2.0 * M_PI / (3.0 * s), fac = pow(h / (2.0 * M_PI), 2);
        for (int k2 = 0; k2 <= maxk2; ++k2) dmemo[k2] = fac * orc2_dhat(ps, kern, lam, l, h * sqrt((double)k2));

#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->fout[b]) continue;
            phi[b] = (cplx *)malloc((size_t)n2 * sizeof(cplx));
            proxy_to_pw2(&ch, proxy[b], h, s, nf, phi[b]);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->fin[b] || t->pcount[b] == 0) continue;
            double cb[2];
            box_center2(t, b, cb);
            cplx *psi = (cplx *)calloc((size_t)n2, sizeof(cplx));
            cplx e0[64], e1[64];
            for (int k = 0; k < 9; ++k) {
                int64_t sb = t->colleague[b * 9 + k];
                if (sb < 0 || !t->fout[sb]) continue;
                double cs[2];
                box_center2(t, sb, cs);
                for (int m = 0; m < nn; ++m) {
                    e0[m] = cexp(I * h * (m - nf) * (cb[0] - cs[0]));
                    e1[m] = cexp(I * h * (m - nf) * (cb[1] - cs[1]));
                }
                for (int a = 0; a < nn; ++a)
                    for (int bb = 0; bb < nn; ++bb) psi[a * nn + bb] += e0[a] * e1[bb] * phi[sb][a * nn + bb];
            }
            for (int a = 0; a < nn; ++a)
                for (int bb = 0; bb < nn; ++bb)
                    psi[a * nn + bb] *= dmemo[(a - nf) * (a - nf) + (bb - nf) * (bb - nf)];
            if (!local[b]) local[b] = (double *)calloc((size_t)p2, sizeof(double));
            pw_to_grid2(&ch, psi, h, s, nf, local[b]);
            free(psi);
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = b0; b < b1; ++b) {
            if (!t->leaf[b] || t->pcount[b] == 0) continue;
            double c[2];
            box_center2(t, b, c);
            double u0[64], u1[64];
            for (int64_t i = t->pstart[b]; i < t->pstart[b] + t->pcount[b]; ++i) {
                const double *x = &t->xs[2 * i];
                cheb_interp_row(&ch, 2.0 * (x[0] - c[0]) / s, u0);
                cheb_interp_row(&ch, 2.0 * (x[1] - c[1]) / s, u1);
                double acc = 0.0;
                for (int a = 0; a < p; ++a)
                    for (int bb = 0; bb < p; ++bb) acc += local[b][a * p + bb] * u0[a] * u1[bb];
                res->ufar[i] = acc;
            }
        }
        /* local expansions to the children (Lemma 2.2) */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = b0; b < b1; ++b) {
            if (t->leaf[b] || t->pcount[b] == 0) continue;
            double *tA = (double *)malloc((size_t)p2 * sizeof(double));
            double *tB = (double *)malloc((size_t)p2 * sizeof(double));
            double *AT[2] = {(double *)malloc((size_t)p2 * sizeof(double)),
                             (double *)malloc((size_t)p2 * sizeof(double))};
            for (int sgn = 0; sgn < 2; ++sgn)
                for (int i = 0; i < p; ++i)
                    for (int a = 0; a < p; ++a) AT[sgn][i * p + a] = ch.A[sgn][a * p + i];
            int dims[2] = {p, p};
            for (int k = 0; k < 4; ++k) {
                int64_t cbx = t->child0[b] + k;
                if (t->pcount[cbx] == 0) continue;
                int o[2];
                child_bits2(t, cbx, o);
                mode_real2(local[b], dims, 1, AT[o[1]], p, tA);
                mode_real2(tA, dims, 0, AT[o[0]], p, tB);
                local[cbx] = (double *)malloc((size_t)p2 * sizeof(double));
                memcpy(local[cbx], tB, (size_t)p2 * sizeof(double));
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
    free(dmemo);

    /* ---- Steps 4-5: residual sums and the r = 0 correction */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t T = 0; T < nbox; ++T) {
        if (!t->terminal[T] || t->pcount[T] == 0) continue;
        const int l = t->level[T];
        const double s = ldexp(1.0, -l);
        const double m0 = sp.self[l] + C;
        int64_t lists[9 + 3][2];
        int nl = 0;
        for (int k = 0; k < 9; ++k) {
            int64_t cb = t->colleague[T * 9 + k];
            if (cb < 0 || t->pcount[cb] == 0) continue;
            lists[nl][0] = t->pstart[cb];
            lists[nl][1] = t->pstart[cb] + t->pcount[cb];
            nl++;
        }
        if (t->leaf[T])
            for (int k = 0; k < t->ncoarse[T]; ++k) {
                int64_t cb = t->coarse[T * 3 + k];
                if (t->pcount[cb] == 0) continue;
                lists[nl][0] = t->pstart[cb];
                lists[nl][1] = t->pstart[cb] + t->pcount[cb];
                nl++;
            }
        for (int64_t j = t->pstart[T]; j < t->pstart[T] + t->pcount[T]; ++j) {
            const double *y = &t->xs[2 * j];
            for (int li = 0; li < nl; ++li)
                for (int64_t i = lists[li][0]; i < lists[li][1]; ++i) {
                    const double *x = &t->xs[2 * i];
                    double dx = x[0] - y[0], dy = x[1] - y[1];
                    double r = sqrt(dx * dx + dy * dy);
                    double contrib;
                    if (r == 0.0) contrib = -m0 * q[j];
                    else if (r < s) contrib = orc2_residual(&sp, l, r) * q[j];
                    else continue;
#pragma omp atomic
                    res->ures[i] += contrib;
                }
        }
    }

    for (int64_t i = 0; i < n; ++i) res->u[t->perm[i]] = res->ufar[i] + res->ures[i];

    if (keep) {
        res->proxy = proxy;
        res->local = local;
    } else {
        for (int64_t b = 0; b < nbox; ++b) { free(proxy[b]); free(local[b]); }
        free(proxy);
        free(local);
    }
    orc2_split_free(&sp);
    cheb_free(&ch);
    free(q);
    return 0;
}

void orc_direct2(int kern, double lam, int64_t n, const double *pts, const double *q, int64_t nt,
                 const int64_t *tidx, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tidx[t];
        double s = 0.0, comp = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pts[2 * i] - pts[2 * j], dy = pts[2 * i + 1] - pts[2 * j + 1];
            double r = sqrt(dx * dx + dy * dy);
            if (r == 0.0) continue;
            double v = q[j] * orc2_kernel(kern, lam, r), tsum = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - tsum) + v;
            else comp += (v - tsum) + s;
            s = tsum;
        }
        out[t] = s + comp;
    }
}
