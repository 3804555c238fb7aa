/* cheb.h -- Chebyshev grid helpers shared by the 3-D and 2-D oracle drivers.
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#ifndef DMK_ORACLE_CHEB_H
#define DMK_ORACLE_CHEB_H

/* ---------------------------------------------------------- Chebyshev */
typedef struct {
    int p;
    double *x;     /* nodes r_i = cos(pi (i - 1/2) / p), i = 1..p          */
    double *vinv;  /* V^{-1}, V(i,j) = T_{j-1}(r_i)  (Sec. 2.1)            */
    double *A[2];  /* A_sigma[a][i] = ell_a((r_i + sigma)/2), sigma = -1,+1 */
} cheb_t;

void cheb_T(int p, double x, double *T);
void cheb_interp_row(const cheb_t *ch, double xi, double *u);
void cheb_init(int p, cheb_t *ch);
void cheb_free(cheb_t *ch);

#endif
