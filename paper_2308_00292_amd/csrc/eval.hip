// Steps 2-5 of the discrete DMK algorithm (Sec. 3.6) on gfx950, FP64.
//
// Stage map (one kernel per stage and level; one workgroup per box):
//   k_gather_q      charges into Morton order
//   k_upward        proxy charges of every F_out box (Step 2): F_out children
//                   are merged with the child->parent anterpolation matrices
//                   (Lemma 2.1); the points of all other children are
//                   anterpolated straight onto the parent grid (Def. 2.1).
//                   Both give the same proxies (Lemma 2.1 is exact), the
//                   second skips proxy grids nobody else reads.
//   k_root_w0       windowed kernel W_0 over the unit box (root only)
//   k_proxy2pw      outgoing plane waves Phi_l(B) of F_out boxes
//                   (eq. outgoingexpansion2), Hermitian half spectrum
//   k_local_init    local values inherited from the parent (Lemma 2.2)
//   k_pwshift       incoming plane waves Psi_l(B) by diagonal translation
//                   from F_out colleagues (eq. diagonaltranslation); with
//                   h_l s_l = 2 pi / 3 the phases are cube roots of unity
//   k_pw2grid       Psi_l(B) -> values on B's Chebyshev grid
//                   (eq. incomingexpansion2)
//   k_leaf_eval     far potential at the targets of each leaf (eq.
//                   farpotential) by tensor Lagrange interpolation
//   k_residual      residual-kernel sums (Step 4) in gather form, including
//                   the r = 0 self correction (Step 5)
//   k_finalize      scale by 1/(4 pi S) and scatter to input order
//
// Data layout in HBM: sorted points as SoA FP64; per-box p^3 arrays with the
// x index slowest, (i*p + j)*p + k; plane waves as [m3][m2][m1] complex
// (interleaved re, im) with m3 = 0..nf (half spectrum) and m1, m2 = -nf..nf.
#include <algorithm>
#include <cmath>

#include "dmk_internal.h"

namespace dmk {

namespace {

constexpr int TPB = 256;
constexpr int MAXP = 18;                 // largest proxy order on the device
constexpr int MAXNPT = (MAXP * MAXP * MAXP + TPB - 1) / TPB;  // owned entries per thread
constexpr int MAXN = 2 * 12 + 1;         // largest plane-wave width (nf <= 12)
constexpr int GSL = 4;                   // m3 slices per group in pw2grid

struct Dev {
    int p, p2, p3, nf, nn, nh, nw, nwn, nwh, gdeg;
    const double *X, *Y, *Z;
    const int32_t *pstart, *pcount, *child0, *parent, *col, *proxy_slot, *local_slot, *psi_slot, *blevel;
    const uint8_t *bflags;
    const double *bcenter;
    const double *c2p, *epw, *ew, *wd0, *ww, *gcheb, *xcheb, *bary;
    double *qs, *proxy, *local, *phi, *psi, *w0vals, *ufar, *ures;
};

// Lagrange basis of the Chebyshev nodes at xi (barycentric formula).
__device__ inline void lagrange_row(const Dev &D, double xi, double *out)
{
    const int p = D.p;
    double den = 0.0;
    int hit = -1;
    for (int a = 0; a < p; ++a) {
        double d = xi - D.xcheb[a];
        if (d == 0.0) hit = a;
        double v = D.bary[a] / d;
        out[a] = v;
        den += v;
    }
    if (hit >= 0) {
        for (int a = 0; a < p; ++a) out[a] = (a == hit) ? 1.0 : 0.0;
        return;
    }
    double inv = 1.0 / den;
    for (int a = 0; a < p; ++a) out[a] *= inv;
}

// Accumulate into the thread's owned entries e = tid + TPB*m of a p^3 grid
// the anterpolation of points [i0, i1) onto the grid of a box with centre c
// and side s.  Uses LDS scratch of at most p^3 doubles (chunks of CH points,
// 3 CH p Lagrange values and CH charges).
__device__ void anterpolate_points(const Dev &D, int64_t i0, int64_t i1, const double *c, double s,
                                   double *sL, double *acc)
{
    const int p = D.p, p2 = D.p2, p3 = D.p3;
    const int CH = min(64, p3 / (3 * p + 1));
    double *Lx = sL, *Ly = Lx + CH * p, *Lz = Ly + CH * p, *qq = Lz + CH * p;
    const double sc = 2.0 / s;
    for (int64_t base = i0; base < i1; base += CH) {
        int cnt = (int)min<int64_t>(CH, i1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < 3 * cnt; t += TPB) {
            int pt = t / 3, d = t % 3;
            int64_t i = base + pt;
            double x = (d == 0) ? D.X[i] : (d == 1) ? D.Y[i] : D.Z[i];
            double xi = (x - c[d]) * sc;
            double row[MAXP];
            lagrange_row(D, xi, row);
            double *dst = (d == 0 ? Lx : d == 1 ? Ly : Lz) + pt * p;
            for (int a = 0; a < p; ++a) dst[a] = row[a];
        }
        for (int t = threadIdx.x; t < cnt; t += TPB) qq[t] = D.qs[base + t];
        __syncthreads();
        for (int m = 0; m < MAXNPT; ++m) {
            int e = threadIdx.x + TPB * m;
            if (e >= p3) break;
            int a0 = e / p2, a1 = (e / p) % p, a2 = e % p;
            double s_ = 0.0;
            for (int pt = 0; pt < cnt; ++pt) s_ += Lx[pt * p + a0] * Ly[pt * p + a1] * (Lz[pt * p + a2] * qq[pt]);
            acc[m] += s_;
        }
    }
}

// ------------------------------------------------------------------ upward
__global__ void __launch_bounds__(TPB) k_upward(Dev D, const int32_t *list)
{
    extern __shared__ double sm[];
    const int p = D.p, p2 = D.p2, p3 = D.p3;
    double *tmp = sm;          // p^3
    double *buf = tmp + p3;    // p^3 (also point scratch)
    double *Am = buf + p3;     // 2 p^2
    const int32_t P = list[blockIdx.x];
    for (int t = threadIdx.x; t < 2 * p2; t += TPB) Am[t] = D.c2p[t];
    double acc[MAXNPT];
    for (int m = 0; m < MAXNPT; ++m) acc[m] = 0.0;
    const double *cP = D.bcenter + 3 * (int64_t)P;
    const double sideP = ldexp(1.0, -D.blevel[P]);
    for (int k = 0; k < 8; ++k) {
        const int32_t C = D.child0[P] + k;
        const int cnt = D.pcount[C];
        if (cnt == 0) continue;
        if (D.bflags[C] & 2) {
            const double *src = D.proxy + (int64_t)D.proxy_slot[C] * p3;
            const double *Ax = Am + ((k >> 2) & 1) * p2, *Ay = Am + ((k >> 1) & 1) * p2, *Az = Am + (k & 1) * p2;
            __syncthreads();
            // z: tmp[i0][i1][a2] = sum_i2 Az[a2][i2] src[i0][i1][i2]
            for (int e = threadIdx.x; e < p3; e += TPB) {
                int r = e / p, a2 = e % p;
                const double *row = src + (int64_t)r * p;
                double s_ = 0.0;
                for (int i = 0; i < p; ++i) s_ += Az[a2 * p + i] * row[i];
                tmp[e] = s_;
            }
            __syncthreads();
            // y: buf[i0][a1][a2] = sum_i1 Ay[a1][i1] tmp[i0][i1][a2]
            for (int e = threadIdx.x; e < p3; e += TPB) {
                int i0 = e / p2, a1 = (e / p) % p, a2 = e % p;
                double s_ = 0.0;
                for (int i = 0; i < p; ++i) s_ += Ay[a1 * p + i] * tmp[i0 * p2 + i * p + a2];
                buf[e] = s_;
            }
            __syncthreads();
            // x: acc[a0][a1][a2] += sum_i0 Ax[a0][i0] buf[i0][a1][a2]
            for (int m = 0; m < MAXNPT; ++m) {
                int e = threadIdx.x + TPB * m;
                if (e >= p3) break;
                int a0 = e / p2, rest = e % p2;
                double s_ = 0.0;
                for (int i = 0; i < p; ++i) s_ += Ax[a0 * p + i] * buf[i * p2 + rest];
                acc[m] += s_;
            }
        } else {
            double c[3] = {cP[0], cP[1], cP[2]};
            anterpolate_points(D, D.pstart[C], D.pstart[C] + cnt, c, sideP, buf, acc);
        }
    }
    double *dst = D.proxy + (int64_t)D.proxy_slot[P] * p3;
    for (int m = 0; m < MAXNPT; ++m) {
        int e = threadIdx.x + TPB * m;
        if (e < p3) dst[e] = acc[m];
    }
}

// ------------------------------------------- proxies -> plane waves (LDS)
// rho (p^3, LDS) -> out[m3][m2][m1] (complex, global), multiplied by wts
// (half spectrum, may be null).  E is [n][p] complex with row m+nf.
__device__ void proxy_to_pw(const Dev &D, const double *rho, const double *E, int n, int nh, double *Abuf,
                            double *Bbuf, int gmax, double *out, const double *wts)
{
    const int p = D.p, p2 = D.p2, nf = (n - 1) / 2;
    // A[m3][j1][j2] = sum_j3 E[m3][j3] rho[j1][j2][j3]
    for (int e = threadIdx.x; e < nh * p2; e += TPB) {
        int m3 = e / p2, r = e % p2;
        const double *Er = E + 2 * (int64_t)(m3 + nf) * p;
        const double *row = rho + r * p;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < p; ++j) {
            re += Er[2 * j] * row[j];
            im += Er[2 * j + 1] * row[j];
        }
        Abuf[2 * e] = re;
        Abuf[2 * e + 1] = im;
    }
    __syncthreads();
    for (int g0 = 0; g0 < nh; g0 += gmax) {
        int g = min(gmax, nh - g0);
        // B[m3][j1][m2] = sum_j2 E[m2][j2] A[m3][j1][j2]
        for (int e = threadIdx.x; e < g * p * n; e += TPB) {
            int mm = e / (p * n), j1 = (e / n) % p, m2 = e % n;
            const double *Ar = Abuf + 2 * ((int64_t)(g0 + mm) * p2 + j1 * p);
            const double *Er = E + 2 * (int64_t)m2 * p;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < p; ++j) {
                double er = Er[2 * j], ei = Er[2 * j + 1], ar = Ar[2 * j], ai = Ar[2 * j + 1];
                re += er * ar - ei * ai;
                im += er * ai + ei * ar;
            }
            Bbuf[2 * e] = re;
            Bbuf[2 * e + 1] = im;
        }
        __syncthreads();
        // out[m3][m2][m1] = sum_j1 E[m1][j1] B[m3][j1][m2]
        for (int e = threadIdx.x; e < g * n * n; e += TPB) {
            int mm = e / (n * n), m2 = (e / n) % n, m1 = e % n;
            const double *Er = E + 2 * (int64_t)m1 * p;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < p; ++j) {
                const double *b = Bbuf + 2 * ((int64_t)mm * p * n + j * n + m2);
                double er = Er[2 * j], ei = Er[2 * j + 1];
                re += er * b[0] - ei * b[1];
                im += er * b[1] + ei * b[0];
            }
            int64_t o = ((int64_t)(g0 + mm) * n + m2) * n + m1;
            double w = wts ? wts[o] : 1.0;
            out[2 * o] = re * w;
            out[2 * o + 1] = im * w;
        }
        __syncthreads();
    }
}

// psi[m3][m2][m1] (global, half spectrum) -> acc (owned grid entries) +=
// Re sum_m exp(+i theta m.x_j) psi[m], E as above (its conjugate is used).
__device__ void pw_to_grid(const Dev &D, const double *psi, const double *E, int n, int nh, double *Sbuf,
                           double *C1, double *C2, double *acc)
{
    const int p = D.p, p2 = D.p2, p3 = D.p3;
    for (int g0 = 0; g0 < nh; g0 += GSL) {
        int g = min(GSL, nh - g0);
        __syncthreads();
        for (int e = threadIdx.x; e < g * n * n; e += TPB) {
            Sbuf[2 * e] = psi[2 * ((int64_t)g0 * n * n + e)];
            Sbuf[2 * e + 1] = psi[2 * ((int64_t)g0 * n * n + e) + 1];
        }
        __syncthreads();
        // C1[m3][m2][j1] = sum_m1 conj(E[m1][j1]) S[m3][m2][m1]
        for (int e = threadIdx.x; e < g * n * p; e += TPB) {
            int mm = e / (n * p), m2 = (e / p) % n, j1 = e % p;
            const double *Sr = Sbuf + 2 * ((int64_t)mm * n * n + m2 * n);
            double re = 0.0, im = 0.0;
            for (int m1 = 0; m1 < n; ++m1) {
                double er = E[2 * (m1 * p + j1)], ei = -E[2 * (m1 * p + j1) + 1];
                double sr = Sr[2 * m1], si = Sr[2 * m1 + 1];
                re += er * sr - ei * si;
                im += er * si + ei * sr;
            }
            C1[2 * e] = re;
            C1[2 * e + 1] = im;
        }
        __syncthreads();
        // C2[m3][j1][j2] = sum_m2 conj(E[m2][j2]) C1[m3][m2][j1]
        for (int e = threadIdx.x; e < g * p2; e += TPB) {
            int mm = e / p2, j1 = (e / p) % p, j2 = e % p;
            double re = 0.0, im = 0.0;
            for (int m2 = 0; m2 < n; ++m2) {
                double er = E[2 * (m2 * p + j2)], ei = -E[2 * (m2 * p + j2) + 1];
                const double *c = C1 + 2 * ((int64_t)mm * n * p + m2 * p + j1);
                re += er * c[0] - ei * c[1];
                im += er * c[1] + ei * c[0];
            }
            C2[2 * e] = re;
            C2[2 * e + 1] = im;
        }
        __syncthreads();
        // acc[j1][j2][j3] += sum_m3 w_m3 Re(conj(E[m3][j3]) C2[m3][j1][j2])
        const int nf = (n - 1) / 2;
        for (int m = 0; m < MAXNPT; ++m) {
            int e = threadIdx.x + TPB * m;
            if (e >= p3) break;
            int r = e / p, j3 = e % p;
            double s_ = 0.0;
            for (int mm = 0; mm < g; ++mm) {
                int m3 = g0 + mm;
                double er = E[2 * ((m3 + nf) * p + j3)], ei = -E[2 * ((m3 + nf) * p + j3) + 1];
                const double *c = C2 + 2 * ((int64_t)mm * p2 + r);
                double v = er * c[0] - ei * c[1];
                s_ += (m3 == 0) ? v : 2.0 * v;
            }
            acc[m] += s_;
        }
    }
}

__global__ void __launch_bounds__(TPB) k_proxy2pw(Dev D, const int32_t *list, int64_t slot0)
{
    extern __shared__ double sm[];
    const int p3 = D.p3;
    double *rho = sm;                         // p^3
    double *E = rho + p3;                     // nn*p*2
    double *A = E + 2 * D.nn * D.p;           // nh*p^2*2
    const int32_t B = list[blockIdx.x];
    const double *src = D.proxy + (int64_t)D.proxy_slot[B] * p3;
    for (int t = threadIdx.x; t < p3; t += TPB) rho[t] = src[t];
    for (int t = threadIdx.x; t < 2 * D.nn * D.p; t += TPB) E[t] = D.epw[t];
    __syncthreads();
    int64_t slot = D.proxy_slot[B] - slot0;
    double *out = D.phi + 2 * slot * (int64_t)D.nh * D.nn * D.nn;
    // B groups reuse the rho region once A is formed
    int gmax = max(1, p3 / (2 * D.p * D.nn));
    proxy_to_pw(D, rho, E, D.nn, D.nh, A, rho, gmax, out, nullptr);
}

__global__ void __launch_bounds__(TPB) k_root_w0(Dev D, int root_fout, double *scratch)
{
    extern __shared__ double sm[];
    const int p3 = D.p3;
    double *E = sm;                     // nwn*p*2
    double *rho = E + 2 * D.nn * D.p;   // p^3
    double *A = rho + p3;               // nh*p^2*2 (point scratch while anterpolating)
    double acc[MAXNPT];
    for (int m = 0; m < MAXNPT; ++m) acc[m] = 0.0;
    if (root_fout) {
        const double *src = D.proxy + (int64_t)D.proxy_slot[0] * p3;
        for (int m = 0; m < MAXNPT; ++m) {
            int e = threadIdx.x + TPB * m;
            if (e < p3) acc[m] = src[e];
        }
    } else {
        double c[3] = {0.0, 0.0, 0.0};
        anterpolate_points(D, 0, D.pcount[0], c, 1.0, A, acc);
    }
    __syncthreads();
    for (int m = 0; m < MAXNPT; ++m) {
        int e = threadIdx.x + TPB * m;
        if (e < p3) rho[e] = acc[m];
    }
    for (int t = threadIdx.x; t < 2 * D.nwn * D.p; t += TPB) E[t] = D.ew[t];
    __syncthreads();
    int gmax = max(1, p3 / (2 * D.p * D.nwn));
    proxy_to_pw(D, rho, E, D.nwn, D.nwh, A, rho, gmax, scratch, D.ww);
    __threadfence_block();
    __syncthreads();
    for (int m = 0; m < MAXNPT; ++m) acc[m] = 0.0;
    double *Sb = rho;
    double *C1 = Sb + 2 * GSL * D.nwn * D.nwn;
    double *C2 = C1 + 2 * GSL * D.nwn * D.p;
    pw_to_grid(D, scratch, E, D.nwn, D.nwh, Sb, C1, C2, acc);
    for (int m = 0; m < MAXNPT; ++m) {
        int e = threadIdx.x + TPB * m;
        if (e < p3) D.w0vals[e] = acc[m];
    }
}

// ------------------------------------------------------------- downward
__global__ void __launch_bounds__(TPB) k_local_init(Dev D, const int32_t *list, int level)
{
    extern __shared__ double sm[];
    const int p = D.p, p2 = D.p2, p3 = D.p3;
    const int32_t B = list[blockIdx.x];
    double *dst = D.local + (int64_t)D.local_slot[B] * p3;
    if (level == 0) {
        for (int e = threadIdx.x; e < p3; e += TPB) dst[e] = D.w0vals[e];
        return;
    }
    double *tmp = sm, *buf = tmp + p3, *Am = buf + p3;
    for (int t = threadIdx.x; t < 2 * p2; t += TPB) Am[t] = D.c2p[t];
    __syncthreads();
    const int32_t Pb = D.parent[B];
    const int k = B - D.child0[Pb];
    const double *src = D.local + (int64_t)D.local_slot[Pb] * p3;
    const double *Ax = Am + ((k >> 2) & 1) * p2, *Ay = Am + ((k >> 1) & 1) * p2, *Az = Am + (k & 1) * p2;
    // z: tmp[a0][a1][i2] = sum_a2 Az[a2][i2] src[a0][a1][a2]
    for (int e = threadIdx.x; e < p3; e += TPB) {
        int r = e / p, i2 = e % p;
        const double *row = src + (int64_t)r * p;
        double s_ = 0.0;
        for (int a = 0; a < p; ++a) s_ += Az[a * p + i2] * row[a];
        tmp[e] = s_;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < p3; e += TPB) {
        int a0 = e / p2, i1 = (e / p) % p, i2 = e % p;
        double s_ = 0.0;
        for (int a = 0; a < p; ++a) s_ += Ay[a * p + i1] * tmp[a0 * p2 + a * p + i2];
        buf[e] = s_;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < p3; e += TPB) {
        int i0 = e / p2, rest = e % p2;
        double s_ = 0.0;
        for (int a = 0; a < p; ++a) s_ += Ax[a * p + i0] * buf[a * p2 + rest];
        dst[e] = s_;
    }
}

__global__ void __launch_bounds__(TPB) k_pwshift(Dev D, const int32_t *list, int64_t fout_slot0, double wscale)
{
    __shared__ int32_t src_slot[27];
    __shared__ int8_t dl[27][3];
    __shared__ int nsrc;
    const int32_t B = list[blockIdx.x];
    if (threadIdx.x == 0) {
        int c = 0;
        for (int k = 0; k < 27; ++k) {
            int32_t S = D.col[(int64_t)B * 27 + k];
            if (S >= 0 && (D.bflags[S] & 2)) {
                src_slot[c] = (int32_t)(D.proxy_slot[S] - fout_slot0);
                // c_S - c_B = delta s_l with delta = offset of the colleague
                dl[c][0] = (int8_t)(k / 9 - 1);
                dl[c][1] = (int8_t)((k / 3) % 3 - 1);
                dl[c][2] = (int8_t)(k % 3 - 1);
                c++;
            }
        }
        nsrc = c;
    }
    __syncthreads();
    const int nn = D.nn, nf = D.nf;
    const int64_t nm = (int64_t)D.nh * nn * nn;
    double *out = D.psi + 2 * (int64_t)D.psi_slot[B] * nm;
    // exp(i h m.(c_B - c_S)) = exp(-2 pi i (m.delta)/3) = w^{-(m.delta mod 3)}
    const double c3 = -0.5, s3 = 0.86602540378443864676;
    for (int64_t e = threadIdx.x; e < nm; e += TPB) {
        int m3 = (int)(e / (nn * nn)), m2 = (int)((e / nn) % nn) - nf, m1 = (int)(e % nn) - nf;
        double re = 0.0, im = 0.0;
        for (int k = 0; k < nsrc; ++k) {
            const double *f = D.phi + 2 * ((int64_t)src_slot[k] * nm + e);
            int t = (m1 * dl[k][0] + m2 * dl[k][1] + m3 * dl[k][2]) % 3;
            if (t < 0) t += 3;
            double fr = f[0], fi = f[1];
            if (t == 0) { re += fr; im += fi; }
            else if (t == 1) { re += c3 * fr + s3 * fi; im += c3 * fi - s3 * fr; }   // * (c3 - i s3)
            else { re += c3 * fr - s3 * fi; im += c3 * fi + s3 * fr; }               // * (c3 + i s3)
        }
        double w = D.wd0[e] * wscale;
        out[2 * e] = re * w;
        out[2 * e + 1] = im * w;
    }
}

__global__ void __launch_bounds__(TPB) k_pw2grid(Dev D, const int32_t *list)
{
    extern __shared__ double sm[];
    const int p = D.p, p3 = D.p3, nn = D.nn;
    double *E = sm;
    double *Sb = E + 2 * nn * p;
    double *C1 = Sb + 2 * GSL * nn * nn;
    double *C2 = C1 + 2 * GSL * nn * p;
    const int32_t B = list[blockIdx.x];
    for (int t = threadIdx.x; t < 2 * nn * p; t += TPB) E[t] = D.epw[t];
    double *v = D.local + (int64_t)D.local_slot[B] * p3;
    double acc[MAXNPT];
    for (int m = 0; m < MAXNPT; ++m) {
        int e = threadIdx.x + TPB * m;
        acc[m] = (e < p3) ? v[e] : 0.0;
    }
    const double *psi = D.psi + 2 * (int64_t)D.psi_slot[B] * D.nh * nn * nn;
    pw_to_grid(D, psi, E, nn, D.nh, Sb, C1, C2, acc);
    for (int m = 0; m < MAXNPT; ++m) {
        int e = threadIdx.x + TPB * m;
        if (e < p3) v[e] = acc[m];
    }
}

__global__ void __launch_bounds__(TPB) k_leaf_eval(Dev D, const int32_t *list)
{
    extern __shared__ double sm[];
    const int p = D.p, p2 = D.p2, p3 = D.p3;
    const int CH = 64;
    double *v = sm;
    double *Lx = v + p3, *Ly = Lx + CH * p, *Lz = Ly + CH * p, *part = Lz + CH * p;
    const int32_t B = list[blockIdx.x];
    const double *src = D.local + (int64_t)D.local_slot[B] * p3;
    for (int t = threadIdx.x; t < p3; t += TPB) v[t] = src[t];
    const double *c = D.bcenter + 3 * (int64_t)B;
    const int64_t i0 = D.pstart[B], i1 = i0 + D.pcount[B];
    const double s = ldexp(1.0, -D.blevel[B]);
    const double sc = 2.0 / s;
    for (int64_t base = i0; base < i1; base += CH) {
        int cnt = (int)min<int64_t>(CH, i1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < 3 * cnt; t += TPB) {
            int pt = t / 3, d = t % 3;
            int64_t i = base + pt;
            double x = (d == 0) ? D.X[i] : (d == 1) ? D.Y[i] : D.Z[i];
            double row[MAXP];
            lagrange_row(D, (x - c[d]) * sc, row);
            double *dst = (d == 0 ? Lx : d == 1 ? Ly : Lz) + pt * p;
            for (int a = 0; a < p; ++a) dst[a] = row[a];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cnt * p; t += TPB) {
            int j1 = t / cnt, pt = t % cnt;
            const double *ly = Ly + pt * p, *lz = Lz + pt * p;
            double s1 = 0.0;
            for (int j2 = 0; j2 < p; ++j2) {
                const double *row = v + j1 * p2 + j2 * p;
                double s2 = 0.0;
                for (int j3 = 0; j3 < p; ++j3) s2 += row[j3] * lz[j3];
                s1 += ly[j2] * s2;
            }
            part[pt * p + j1] = Lx[pt * p + j1] * s1;
        }
        __syncthreads();
        for (int pt = threadIdx.x; pt < cnt; pt += TPB) {
            double s_ = 0.0;
            for (int j1 = 0; j1 < p; ++j1) s_ += part[pt * p + j1];
            D.ufar[base + pt] = s_;
        }
    }
}

// ------------------------------------------------------------- residual
__global__ void __launch_bounds__(TPB) k_residual(Dev D, const int32_t *leaves, const int32_t *nl_off,
                                                  const int32_t *nl_src, const int32_t *blevel)
{
    __shared__ double sx[TPB], sy[TPB], sz[TPB], sq[TPB];
    __shared__ double part[TPB];
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = D.pstart[B];
    const int nt = D.pcount[B];
    const int tch = (nt <= 32) ? 32 : 64;
    const int nsplit = TPB / tch;
    const int tl = threadIdx.x % tch, split = threadIdx.x / tch;
    const int32_t l0 = nl_off[blockIdx.x], l1 = nl_off[blockIdx.x + 1];
    const int deg = D.gdeg;
    for (int tbase = 0; tbase < nt; tbase += tch) {
        const bool active = (tbase + tl) < nt;
        const int64_t it = t0 + tbase + (active ? tl : 0);
        const double xt = D.X[it], yt = D.Y[it], zt = D.Z[it];
        double acc = 0.0;
        for (int li = l0; li < l1; ++li) {
            const int32_t T = nl_src[li];
            const int lev = blevel[T];
            const double inv_s = ldexp(1.0, lev), inv_s2 = inv_s * inv_s, s2 = 1.0 / inv_s2;
            const int64_t j0 = D.pstart[T];
            const int ns = D.pcount[T];
            for (int jb = 0; jb < ns; jb += TPB) {
                int cnt = min(TPB, ns - jb);
                __syncthreads();
                if (threadIdx.x < cnt) {
                    int64_t j = j0 + jb + threadIdx.x;
                    sx[threadIdx.x] = D.X[j];
                    sy[threadIdx.x] = D.Y[j];
                    sz[threadIdx.x] = D.Z[j];
                    sq[threadIdx.x] = D.qs[j];
                }
                __syncthreads();
                for (int j = split; j < cnt; j += nsplit) {
                    double dx = xt - sx[j], dy = yt - sy[j], dz = zt - sz[j];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < s2) {
                        double u = 2.0 * r2 * inv_s2 - 1.0;
                        // Clenshaw for g(t) = Phi(sqrt t)/sqrt t, t = r^2/s^2
                        double b1 = 0.0, b2 = 0.0;
                        for (int k = deg; k >= 1; --k) {
                            double b0 = D.gcheb[k] + 2.0 * u * b1 - b2;
                            b2 = b1;
                            b1 = b0;
                        }
                        double g = D.gcheb[0] + u * b1 - b2;
                        double rinv = (r2 > 0.0) ? rsqrt(r2) : 0.0;
                        acc += sq[j] * (rinv - g * inv_s);
                    }
                }
            }
        }
        __syncthreads();
        part[threadIdx.x] = acc;
        __syncthreads();
        if (split == 0 && active) {
            double s_ = 0.0;
            for (int k = 0; k < nsplit; ++k) s_ += part[k * tch + tl];
            D.ures[t0 + tbase + tl] = s_;
        }
    }
}

__global__ void k_gather_q(const double *charges, const int32_t *perm, int64_t n, double *qs)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) qs[i] = charges[perm[i]];
}

__global__ void k_finalize(const double *ufar, const double *ures, const int32_t *perm, int64_t n, double scale,
                           double *pot, double *farp, double *nearp)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    double f = ufar[i] * scale, r = ures[i] * scale;
    if (pot) pot[j] = f + r;
    if (farp) farp[j] = f;
    if (nearp) nearp[j] = r;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

size_t lds_upward(const Plan *P) { return (size_t)(2 * P->p * P->p * P->p + 2 * P->p * P->p) * sizeof(double); }
size_t lds_p2pw(const Plan *P)
{
    const Tables &t = P->tab;
    return (size_t)(t.p * t.p * t.p + 2 * t.nn * t.p + 2 * t.nh * t.p * t.p) * sizeof(double);
}
size_t lds_local(const Plan *P) { return lds_upward(P); }
size_t lds_pw2grid(const Plan *P)
{
    const Tables &t = P->tab;
    return (size_t)(2 * t.nn * t.p + 2 * GSL * t.nn * t.nn + 2 * GSL * t.nn * t.p + 2 * GSL * t.p * t.p) *
           sizeof(double);
}
size_t lds_root(const Plan *P)
{
    const Tables &t = P->tab;
    size_t a = lds_p2pw(P);
    size_t b = (size_t)(2 * t.nn * t.p + 2 * GSL * (t.nwn * t.nwn + t.nwn * t.p + t.p * t.p)) * sizeof(double);
    return std::max(a, b);
}
size_t lds_leaf(const Plan *P)
{
    return (size_t)(P->p * P->p * P->p + 4 * 64 * P->p) * sizeof(double);
}

Dev make_dev(Plan *P)
{
    Dev D;
    const Tables &t = P->tab;
    D.p = t.p; D.p2 = t.p * t.p; D.p3 = t.p * t.p * t.p;
    D.nf = t.nf; D.nn = t.nn; D.nh = t.nh; D.nw = t.nw; D.nwn = t.nwn; D.nwh = t.nwh; D.gdeg = t.gdeg;
    D.X = P->X; D.Y = P->Y; D.Z = P->Z;
    D.pstart = P->pstart; D.pcount = P->pcount; D.child0 = P->child0; D.parent = P->parent; D.col = P->colleague;
    D.proxy_slot = P->proxy_slot; D.local_slot = P->local_slot; D.psi_slot = P->psi_slot; D.blevel = P->blevel;
    D.bflags = P->bflags; D.bcenter = P->bcenter;
    D.c2p = P->d_c2p; D.epw = P->d_epw; D.ew = P->d_ew; D.wd0 = P->d_wd0; D.ww = P->d_ww;
    D.gcheb = P->d_gcheb; D.xcheb = P->d_xcheb; D.bary = P->d_bary;
    D.qs = P->qs; D.proxy = P->proxy; D.local = P->local; D.phi = P->phi; D.psi = P->psi;
    D.w0vals = P->w0vals; D.ufar = P->ufar; D.ures = P->ures;
    return D;
}

bool g_attr_done = false;
void set_lds_attrs(const Plan *P)
{
    size_t need = std::max({lds_upward(P), lds_p2pw(P), lds_root(P), lds_local(P), lds_pw2grid(P), lds_leaf(P)});
    int dev = 0, lim = 0;
    DMK_HIP(hipGetDevice(&dev));
    DMK_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if ((size_t)lim < need)
        throw Error{DMK_ERR_UNSUPPORTED, "device LDS per workgroup (" + std::to_string(lim) + " B) below the " +
                                             std::to_string(need) + " B the stages need"};
    if (g_attr_done) return;
    const int maxlds = lim;
    DMK_HIP(hipFuncSetAttribute((const void *)k_upward, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    DMK_HIP(hipFuncSetAttribute((const void *)k_proxy2pw, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    DMK_HIP(hipFuncSetAttribute((const void *)k_root_w0, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    DMK_HIP(hipFuncSetAttribute((const void *)k_local_init, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    DMK_HIP(hipFuncSetAttribute((const void *)k_pw2grid, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    DMK_HIP(hipFuncSetAttribute((const void *)k_leaf_eval, hipFuncAttributeMaxDynamicSharedMemorySize, maxlds));
    g_attr_done = true;
}

}  // namespace

void upload_tables(Plan *P, hipStream_t s)
{
    const Tables &t = P->tab;
    auto up = [&](const std::vector<double> &v) {
        double *d = (double *)dalloc(P, std::max<size_t>(v.size(), 1) * sizeof(double));
        if (!v.empty()) DMK_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
        return d;
    };
    P->d_c2p = up(t.c2p);
    P->d_epw = up(t.epw);
    P->d_ew = up(t.ew);
    P->d_wd0 = up(t.wd0);
    P->d_ww = up(t.ww);
    P->d_gcheb = up(t.gcheb);
    P->d_xcheb = up(t.xcheb);
    P->d_bary = up(t.bary);
    DMK_HIP(hipStreamSynchronize(s));
}

void alloc_workspace(Plan *P)
{
    const Tables &t = P->tab;
    const int64_t p3 = (int64_t)t.p * t.p * t.p;
    const int64_t nm = (int64_t)t.nh * t.nn * t.nn;
    const int64_t nmw = (int64_t)t.nwh * t.nwn * t.nwn;
    auto al = [&](int64_t cnt) { return (double *)dalloc(P, (size_t)std::max<int64_t>(cnt, 1) * sizeof(double)); };
    P->qs = al(P->n);
    P->ufar = al(P->n);
    P->ures = al(P->n);
    P->proxy = al(P->nfout * p3);
    P->local = al(P->nne * p3);
    P->phi = al(2 * std::max<int64_t>(P->max_fout_level * nm, nmw));
    P->psi = al(2 * P->max_fin_level * nm);
    P->w0vals = al(p3);
}

void run_eval(Plan *P, const double *charges, double *pot, double *far_part, double *near_part, hipStream_t s)
{
    const int64_t n = P->n;
    if (n == 0) return;
    set_lds_attrs(P);
    Dev D = make_dev(P);
    const auto &ll = P->ll;
    const int L = P->nlevels;
    hipLaunchKernelGGL(k_gather_q, dim3(nblk(n)), dim3(TPB), 0, s, charges, P->perm, n, P->qs);
    // Step 2: upward pass, finest level first
    for (int l = L - 1; l >= 0; --l) {
        int64_t m = ll.fout_off[l + 1] - ll.fout_off[l];
        if (m) hipLaunchKernelGGL(k_upward, dim3((unsigned)m), dim3(TPB), lds_upward(P), s, D, P->l_fout + ll.fout_off[l]);
    }
    // root: windowed kernel W_0 (the phi buffer doubles as scratch)
    int root_fout = (ll.fout_off[1] > 0) ? 1 : 0;
    hipLaunchKernelGGL(k_root_w0, dim3(1), dim3(TPB), lds_root(P), s, D, root_fout, P->phi);
    // Step 3: downward pass
    for (int l = 0; l < L; ++l) {
        int64_t nfo = ll.fout_off[l + 1] - ll.fout_off[l];
        int64_t nne = ll.ne_off[l + 1] - ll.ne_off[l];
        int64_t nfi = ll.fin_off[l + 1] - ll.fin_off[l];
        if (nfo) hipLaunchKernelGGL(k_proxy2pw, dim3((unsigned)nfo), dim3(TPB), lds_p2pw(P), s, D, P->l_fout + ll.fout_off[l], ll.fout_off[l]);
        if (nne) hipLaunchKernelGGL(k_local_init, dim3((unsigned)nne), dim3(TPB), lds_local(P), s, D, P->l_ne + ll.ne_off[l], l);
        if (nfi) {
            hipLaunchKernelGGL(k_pwshift, dim3((unsigned)nfi), dim3(TPB), 0, s, D, P->l_fin + ll.fin_off[l], ll.fout_off[l], std::ldexp(1.0, l));
            hipLaunchKernelGGL(k_pw2grid, dim3((unsigned)nfi), dim3(TPB), lds_pw2grid(P), s, D, P->l_fin + ll.fin_off[l]);
        }
    }
    if (P->nleaf) {
        hipLaunchKernelGGL(k_leaf_eval, dim3((unsigned)P->nleaf), dim3(TPB), lds_leaf(P), s, D, P->l_leaf);
        hipLaunchKernelGGL(k_residual, dim3((unsigned)P->nleaf), dim3(TPB), 0, s, D, P->l_leaf, P->nl_off, P->nl_src, P->blevel);
    }
    const double scale = 1.0 / (4.0 * M_PI * P->side);
    hipLaunchKernelGGL(k_finalize, dim3(nblk(n)), dim3(TPB), 0, s, P->ufar, P->ures, P->perm, n, scale, pot, far_part, near_part);
    DMK_HIP(hipGetLastError());
}

}  // namespace dmk
