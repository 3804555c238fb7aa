/*
 * oracle.h -- plain, slow FP64 CPU oracle for the DMK (dual-space multilevel
 * kernel-splitting) point code of Jiang & Greengard, arXiv 2308.00292.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path.
 *
 * Every routine follows a passage of the paper (cited by section, equation,
 * lemma or table) and is written as plain loops in double precision:
 *   - PSWF psi_0^c (Appendix "Prolate spheroidal wave functions of order
 *     zero", eigenfunction of the operator F_c), its constants c_0, c_2,
 *     lambda_0 and the cumulative window Phi (Sec. 3.7, "Optimization of kernel
 *     splitting using prolate spheroidal wave functions").
 *   - The kernel split 1/r = W_0 + sum_l D_l + R_L (Sec. 3.7, eq. newkernels)
 *     and the plane-wave weights (eqs. differencekernelft3, windowedkernelft2,
 *     wlmdef, with the trapezoidal factor h^d).
 *   - The level-restricted adaptive tree, colleagues, coarse neighbours,
 *     flags F_leaf/F_out/F_in (Sec. 3.2 and Sec. 3.5 "The full DMK algorithm
 *     for discrete sources", Step 0).
 *   - Steps 1-5 of that algorithm: proxies, upward pass, plane-wave outgoing
 *     and incoming expansions, local expansions, direct residual sums,
 *     self-interaction correction.
 *   - Direct O(N M) summation with compensated accumulation (eq. laplacesum).
 *
 * Kernels: 3-D Laplace, K(r) = 1/(4 pi r), and 3-D Yukawa e^{-lambda r}/(4 pi r)
 * (yuk3.c); 2-D log and K_0 (split2.c, dmk2.c).  Sources equal targets; the
 * pair i = j and pairs at distance exactly 0 are excluded from the sum.
 */
#ifndef DMK_ORACLE_H
#define DMK_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- params */
typedef struct {
    double tol;    /* requested precision                              */
    double c;      /* PSWF bandwidth parameter                         */
    int    nf;     /* plane-wave half width for D_l (N_1 = 2 nf + 1)   */
    int    p;      /* Chebyshev proxy order per dimension              */
    int    nw;     /* plane-wave half width for the windowed W_0       */
    double hw;     /* plane-wave spacing for W_0 (root box side 1)     */
} orc_params;

/* Parameters of Table 1 (c, N_1, p); tol 1e-5 uses c = log(1e5), nf = 10,
 * p = 15.  Returns 0 on success, -1 for an unsupported tol. */
int orc_params_for(double tol, orc_params *out);
int orc_params_set(double tol, double c, int nf, int p, int dim, orc_params *out);

/* ------------------------------------------------------------------ PSWF */
#define ORC_PSWF_MAXTERM 96
#define ORC_GL_EXT 256
typedef struct {
    double c;
    int    nterm;                      /* even Legendre terms kept          */
    double coef[ORC_PSWF_MAXTERM];     /* coefficient of sqrt(k+1/2) P_k, k=2i */
    double chi;                        /* Sturm-Liouville eigenvalue         */
    double psi0;                       /* psi(0)                             */
    double lambda0;                    /* eigenvalue of F_c                  */
    double c0, c2;                     /* int_0^1 psi, int_0^1 x^2 psi       */
    double glx[ORC_GL_EXT], glw[ORC_GL_EXT], glpsi[ORC_GL_EXT];
} orc_pswf;

int    orc_pswf_init(double c, orc_pswf *ps);
double orc_pswf_eval(const orc_pswf *ps, double x);     /* |x| <= 1 series   */
double orc_pswf_eval_ext(const orc_pswf *ps, double x); /* any x, via F_c    */
double orc_pswf_phi(const orc_pswf *ps, double x);      /* Phi(x), x >= 0    */
void   orc_gauss_legendre(int n, double *x, double *w);

/* Kernel split for 1/r (unscaled, root box side s_0 = 1). */
double orc_split_w0(const orc_pswf *ps, double r);
double orc_split_d(const orc_pswf *ps, int l, double r);
double orc_split_r(const orc_pswf *ps, int L, double r);
double orc_split_m0(const orc_pswf *ps, int L);          /* M_L(0)           */
/* Fourier transforms (3-D radial) of D_l and of the windowed W_0. */
double orc_dhat(const orc_pswf *ps, int l, double k);
double orc_w0hat(const orc_pswf *ps, double k);
/* Plane-wave (trapezoidal) approximations evaluated at a 3-D offset x. */
double orc_split_d_pw(const orc_pswf *ps, const orc_params *pr, int l,
                      const double x[3]);
double orc_split_w0_pw(const orc_pswf *ps, const orc_params *pr,
                       const double x[3]);

/* ------------------------------------------------------------------ tree */
typedef struct {
    int      dim;          /* 2 or 3                                         */
    int      bits;         /* key bits per dimension (21 in 3-D, 31 in 2-D)   */
    int      ns;           /* leaf capacity n_s                               */
    int      maxdepth;
    int64_t  n;            /* number of points                                */
    double   center[3];    /* root cube centre (input units)                  */
    double   side;         /* root cube side S (input units)                  */
    int64_t *perm;         /* sorted position -> input index                  */
    uint64_t *key;         /* sorted Morton keys                              */
    double  *xs;           /* sorted normalised coordinates [n][dim]          */
    int      nlevels;      /* levels 0 .. nlevels-1                           */
    int64_t *level_start;  /* [nlevels+1] first box of each level             */
    int64_t  nbox;
    int32_t *level;        /* [nbox]                                          */
    uint64_t *bkey;        /* [nbox] Morton prefix of the box at its level    */
    int64_t *parent;       /* [nbox] (-1 for the root)                        */
    int64_t *child0;       /* [nbox] first of 2^d contiguous children or -1   */
    int64_t *pstart;       /* [nbox] first sorted point                       */
    int64_t *pcount;       /* [nbox] number of points                         */
    uint8_t *leaf, *fout, *fin, *terminal;  /* [nbox] flags                   */
    int64_t *colleague;    /* [nbox][3^d], offset order (dx,dy,dz) lexicographic,
                              -1 when absent; entry 3^d/2 is the box itself    */
    int32_t *ncoarse;      /* [nbox]                                          */
    int64_t *coarse;       /* [nbox][2^d - 1] coarse-neighbour leaves         */
    int32_t *tlevel;       /* [n] level of the terminal box of each sorted pt */
} orc_tree;

/* Builds the tree for n points pts[n][dim] (input order).  Returns 0 on
 * success. */
int  orc_tree_build(int dim, int64_t n, const double *pts, int ns,
                    int maxdepth, orc_tree *t);
void orc_tree_free(orc_tree *t);

/* ------------------------------------------------------------------- DMK */
typedef struct {
    int64_t n;
    double *u;        /* [n] potential, input order                        */
    double *ufar;     /* [n] sorted order, normalised units, no 1/(4 pi S) */
    double *ures;     /* [n] sorted order, residual incl. self correction   */
    /* optional intermediates (keep != 0), indexed by box                    */
    int     p, nf;
    double **proxy;   /* [nbox] -> p^3 proxy charges, NULL if not formed   */
    double **local;   /* [nbox] -> p^3 local values on the box's Chebyshev
                         grid (far potential incl. inherited parts)        */
} orc_dmk_result;

int  orc_dmk_eval(const orc_tree *t, const orc_params *pr, const orc_pswf *ps,
                  const double *charges, int keep, orc_dmk_result *res);
/* The same with a choice of 3-D kernel: ORC_LAP3 1/(4 pi r) (physical-space
 * PSWF split, Sec. 3.7), ORC_YUK3 e^{-lambda r}/(4 pi r) (Fourier-space
 * PSWF split, Sec. 4.6; lam in input units, lam S >= 1e-3; see yuk3.c) or
 * ORC_POW3 1/r^2 (PSWF power-function split, Sec. 4.5; see pow2.c). */
enum { ORC_LAP3 = 0, ORC_YUK3 = 1, ORC_POW3 = 2 };
int  orc_dmk_eval_k(const orc_tree *t, const orc_params *pr, const orc_pswf *ps, int kern, double lam,
                    const double *charges, int keep, orc_dmk_result *res);

/* ---- 3-D Yukawa split (yuk3.c); lam in root-box units (lambda S) */
#define ORC3_DEG 47   /* Chebyshev degree (in x^2) of the mollified-kernel tables */
typedef struct {
    double  lam;
    int     nlev, deg;
    double *coef;     /* [nlev][deg+1] m_mu(x), x = r/s_l, series in 2x^2 - 1 */
    double *self;     /* [nlev] M_l(0)                                        */
} orc_split3;
double orc_y3_dhat(const orc_pswf *ps, double lam, int l, double k);
double orc_y3_that(double lam, double k);   /* transform of K cut at (1+sqrt 3) */
double orc_y3_w0hat(const orc_pswf *ps, double lam, double k);
double orc_y3_smooth_quad(const orc_pswf *ps, double mu, double x);  /* m_mu(x) */
int    orc_y3_split_init(const orc_pswf *ps, double lam, int nlev, orc_split3 *sp);
void   orc_y3_split_free(orc_split3 *sp);
double orc_y3_smooth(const orc_split3 *sp, int l, double x);
double orc_y3_residual(const orc_split3 *sp, int l, double r);  /* r > 0, root units */
double orc_y3_d_pw(const orc_pswf *ps, const orc_params *pr, double lam, int l, const double x[3]);
double orc_y3_w0_pw(const orc_pswf *ps, const orc_params *pr, double lam, const double x[3]);
void   orc_direct_yuk3(double lam, int64_t n, const double *pts, const double *q, int64_t nt,
                       const int64_t *tidx, double *out);  /* lam in input units */

/* ---- 3-D 1/r^2 split (pow2.c), root-box units */
#define ORC_P2_NC 48
typedef struct {
    const orc_pswf *ps;
    double c1;                  /* int_0^1 t psi(t) dt                  */
    double coef[ORC_P2_NC];     /* Phi(x)/x^2, series in 2x^2 - 1       */
} orc_pow2;
double orc_p2_c1(const orc_pswf *ps);
double orc_p2_phi_quad(const orc_pswf *ps, double x);   /* Phi by its integral */
int    orc_p2_init(const orc_pswf *ps, orc_pow2 *tb);
double orc_p2_phi(const orc_pow2 *tb, double x);
double orc_p2_m0(const orc_pow2 *tb, int L);
double orc_p2_d(const orc_pow2 *tb, int l, double r);
double orc_p2_r(const orc_pow2 *tb, int L, double r);
double orc_p2_w0(const orc_pow2 *tb, double r);          /* windowed M_0     */
double orc_p2_dhat(const orc_pow2 *tb, int l, double k);
double orc_p2_w0hat(const orc_pow2 *tb, double k);
double orc_p2_d_pw(const orc_pow2 *tb, const orc_params *pr, int l, const double x[3]);
double orc_p2_w0_pw(const orc_pow2 *tb, const orc_params *pr, const double x[3]);
void   orc_direct_pow2(int64_t n, const double *pts, const double *q, int64_t nt, const int64_t *tidx,
                       double *out);
void orc_dmk_result_free(const orc_tree *t, orc_dmk_result *res);

/* Direct sum u_i = sum_{j != i, r_ij > 0} q_j / (4 pi r_ij) for the targets
 * listed in tidx (input indices); compensated (Neumaier) accumulation. */
void orc_direct(int64_t n, const double *pts, const double *q,
                int64_t nt, const int64_t *tidx, double *out);

/* Convenience: full pipeline (params, PSWF, tree, DMK) in one call; the
 * plan/eval wall times in seconds are returned in times[0..1]. */
int orc_dmk_run(int64_t n, const double *pts, const double *q, double tol,
                int ns, int maxdepth, double *u, double *times);

int orc_num_threads(void);
int orc_set_threads(int n);

/* ------------------------------------------------------------------- 2-D
 * Kernels (input units): ORC_LOG2 K(r) = -log(r)/(2 pi); ORC_YUK2 K(r) =
 * K_0(lambda r).  Split in Fourier space (Sec. 4.6, eq. yukawaPSWFkernels),
 * windowed root kernel (Sec. 4.7); see split2.c. */
enum { ORC_LOG2 = 0, ORC_YUK2 = 1 };
#define ORC2_DEG 47   /* Chebyshev degree (in x^2) of the residual tables */

double orc_bessel_k0(double x);
double orc_bessel_k1(double x);
double orc2_kernel(int kern, double lam, double r);
/* Table 1 (c, nf, p); root window spacing hw = 2 pi/(3 + sqrt 2) */
int    orc_params2_for(double tol, orc_params *out);
/* transforms for root side 1; lam is the scaled Yukawa parameter */
double orc2_dhat(const orc_pswf *ps, int kern, double lam, int l, double k);
double orc2_w0hat(const orc_pswf *ps, int kern, double lam, double k);
/* smooth part of the residual by quadrature (definition): log m(x); K_0
 * M_l(x s_l) with mu = lam s_l */
double orc2_smooth_quad(const orc_pswf *ps, int kern, double mu, double x);
typedef struct {
    int     kern;
    double  lam;      /* scaled Yukawa parameter                            */
    int     nlev, deg;
    double *coef;     /* [nlev][deg+1] Chebyshev coefficients in 2(r/s_l)^2-1 */
    double *self;     /* [nlev] M_l(0), the r = 0 limit of the far field    */
} orc_split2;
int    orc2_split_init(const orc_pswf *ps, int kern, double lam, int nlev, orc_split2 *sp);
void   orc2_split_free(orc_split2 *sp);
double orc2_smooth(const orc_split2 *sp, int l, double x);
double orc2_residual(const orc_split2 *sp, int l, double r);  /* r > 0 */
double orc2_d_pw(const orc_pswf *ps, const orc_params *pr, int kern, double lam, int l,
                 const double x[2]);
double orc2_w0_pw(const orc_pswf *ps, const orc_params *pr, int kern, double lam,
                  const double x[2]);

/* DMK in 2-D on a 2-D tree; lam in input units.  ufar/ures are in the
 * scaled (root side 1) problem; for the log kernel the constant
 * -log(S)/(2 pi) of the unit change is carried by ufar (times the total
 * charge) and by the r = 0 correction, so u = ufar + ures in input order. */
int  orc_dmk2_eval(const orc_tree *t, const orc_params *pr, const orc_pswf *ps, int kern,
                   double lam, const double *charges, int keep, orc_dmk_result *res);
/* direct sum over j != i, r_ij > 0, compensated */
void orc_direct2(int kern, double lam, int64_t n, const double *pts, const double *q,
                 int64_t nt, const int64_t *tidx, double *out);

/* --------------------------------------------------------------- volume
 * Volume potential u(x) = int_{B_0} rho(y)/(4 pi |x-y|) dy on the unit cube
 * B_0 = [-1/2,1/2]^3 with the Gaussian multilevel split (Sec. 3.2) and the
 * continuous-source modifications of Sec. 3.6 and Sec. 4.4; see vol.c. */
#define ORC_VFIT_MAX 32
typedef struct {
    double tol;
    int    q;        /* leaf grid: q Chebyshev nodes per axis               */
    double sigma0;   /* Gaussian width at level 0, 1/sqrt(log(1/tol))        */
    int    p, nf;    /* proxy order; plane-wave half width of D_l            */
    int    nw;       /* plane-wave half width of the windowed W_0            */
    double hw;       /* its spacing                                          */
    int    nleg;     /* Gauss-Legendre nodes per axis for proxy charges      */
    double tau_a;    /* t_a = tau_a / (target leaf side)                     */
    int    tpan_gl;  /* Gauss-Legendre nodes per panel in log t              */
    double tpan_w;   /* panel width in log t                                 */
    /* tol 1e-6 takes the PSWF split of Sec. 3.7 (split = 1): D_l and W_0 of
       the point code, and the residual R_L = (1 - Phi(r/s_L))/r as a sum of
       Gaussians -- nfit fitted ones plus the t-quadrature from theta1/s_L */
    int    split;    /* 0: Gaussian split (tol 1e-3); 1: PSWF split          */
    double c;        /* PSWF bandwidth (split 1)                             */
    double theta1;   /* quadrature in t from theta1 / s_L (split 1)          */
    int    nfit;     /* fitted Gaussians (split 1)                           */
    double fit_t[ORC_VFIT_MAX], fit_w[ORC_VFIT_MAX]; /* t s_L and w s_L      */
    double fit_err;  /* max |error| of the fit on its sample grid, x 1/s_L   */
} orc_vparams;
int orc_vparams_for(double tol, int q, orc_vparams *vp);  /* tol 1e-3 or 1e-6 */
/* the part of R_L that the fitted Gaussians stand for, in units of s_L:
   h(x) = (erf(theta1 x) - Phi(x)) / x */
double orc_vfit_target(const orc_vparams *vp, double x);

double orc_gsplit_m(const orc_vparams *vp, int l, double r);   /* erf(r/s_l)/r */
double orc_gsplit_d(const orc_vparams *vp, int l, double r);   /* D_l          */
double orc_gsplit_r(const orc_vparams *vp, int l, double r);   /* R_l          */
double orc_gdhat(const orc_vparams *vp, int l, double k);
double orc_gw0hat(const orc_vparams *vp, double k);
double orc_gsplit_d_pw(const orc_vparams *vp, int l, const double x[3]);
double orc_gsplit_w0_pw(const orc_vparams *vp, const double x[3]);
int    orc_vsog(const orc_vparams *vp, double t_lo, double t_hi, double *t, double *w);
int    orc_vsog_count(const orc_vparams *vp, double t_lo, double t_hi);

/* density callback: out[i] = rho(xyz[3i..3i+2]) for i < n */
typedef void (*orc_density_fn)(int64_t n, const double *xyz, double *out, void *ctx);
typedef struct {
    int      q;
    int64_t  nleaf;
    int32_t *level;  /* [nleaf], leaves in Morton order                      */
    int32_t *ijk;    /* [nleaf][3] integer cell of the leaf at its level      */
} orc_vtree;
/* feat: [nfeat][4] points (x, y, z, h): boxes containing one are split while
 * their side exceeds h */
int  orc_vtree_build(const orc_vparams *vp, double rho_scale, int minlevel, int maxlevel,
                     int nfeat, const double *feat, orc_density_fn fn, void *ctx,
                     orc_vtree *t);  /* maxlevel <= 19 */
void orc_vtree_free(orc_vtree *t);
/* leaf node coordinates [nleaf*q^3][3], leaf-major, node (i,j,k) with k fastest,
 * coordinate c + (s/2) cos(pi (i + 1/2)/q) per axis */
void orc_vol_nodes(const orc_vtree *t, double *xyz);
typedef struct {
    int64_t n;
    double *u, *ufar, *unear, *utail;  /* [n] at the leaf nodes, times 1/(4 pi) */
} orc_vol_result;
int  orc_vol_eval(const orc_vtree *t, const orc_vparams *vp, const double *rho, orc_vol_result *res);
void orc_vol_result_free(orc_vol_result *r);

#ifdef __cplusplus
}
#endif
#endif
