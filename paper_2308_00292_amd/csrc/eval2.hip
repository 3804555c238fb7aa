// Steps 2-5 of the discrete DMK algorithm (Sec. 3.5) in two dimensions on
// gfx950, for the kernel -log(r)/(2 pi) with the Fourier-space PSWF split of
// Sec. 4.6 and the windowed root kernel of Sec. 4.7.  The plan may hold many
// independent problems (a forest, one root per problem); every launch covers
// the boxes of all problems.
//
//   k_upward2    proxy charges (p^2) of each F_out box from its children:
//                F_out children merged with the anterpolation matrices
//                (Lemma 2.1), the points of other children anterpolated
//                straight onto the parent grid (Def. 2.1).
//   k_root2      windowed kernel W_0 of each root on its grid (FP64), plus
//                the constant -log(S_b)/(2 pi) of the unit change times the
//                problem's total charge.
//   k_proxy2pw2  outgoing plane waves Phi_l(B), half spectrum [m1][m2 >= 0].
//   k_pwshift2   incoming plane waves of the 4 children of a parent from the
//                4x4 block of boxes around them, separable in x and y.
//   k_local_pw2  local values of the anchors: interpolation of the nearest
//                anchor ancestor's polynomial (Lemma 2.2) plus the box's own
//                incoming plane waves evaluated on its grid.
//   k_leaf2      far potential at the targets from the anchor polynomial.
//   k_residual2  residual sums -log(r/s)/(2 pi) - m(r/s) for r < s in gather
//                form, with the r = 0 correction.
//   k_finalize2  scatter to input order.
//
// Units: each problem is solved in its own root box [-1/2,1/2]^2 of side
// S_b; -log(S_b r')/(2 pi) = -log(r')/(2 pi) + C_b, C_b = -log(S_b)/(2 pi),
// and a constant kernel is its own far field, so C_b times the total charge
// enters the root values and C_b enters the r = 0 correction.
#include <algorithm>
#include <cmath>

#include "dmk_internal.h"
#include "kfun.h"
#include "lagrange.h"
#include "queue.h"

namespace dmk {

namespace {

constexpr int TPB = 256;

template <typename T>
struct Dev2 {
    int p, nf, nn, nh, nw, nwn, nwh, gdeg, nprob;
    int kern, nlev, ydeg;  // kern: 0 -log(r)/(2 pi), 1 K_0(lambda r)
    const T *ywd, *ycheb;  // K_0: per (problem, level) D_l weights and residual series
    const double *yww, *yself, *ylam;
    double m0;
    const double *X, *Y, *qs, *pside;
    const int32_t *pstart, *pcount, *child0, *parent, *col, *proxy_slot, *local_slot, *psi_slot, *blevel,
        *anchor, *bprob;
    const uint8_t *bflags;
    const uint8_t *anc_read;  // per anchor slot: its values are read by a finer anchor
    const double *bcenter;
    const T *c2p, *epw, *wd0, *gcheb, *gmono, *xcheb, *bary;  // gmono: m(x) as a power series in u = 2x^2 - 1
    const double *ew64, *ww64, *xcheb64, *bary64;
    T *proxy, *local, *phi, *psi, *w0vals;
    double *ufar, *ures;
    int64_t pwstride;  // nn * nh
};

template <typename T>
__device__ inline void lagrange_row(int p, const T *xc, const T *bw, T xi, T *out)
{
    T den = T(0);
    int hit = -1;
    for (int a = 0; a < p; ++a) {
        T d = xi - xc[a];
        if (d == T(0)) hit = a;
        T v = bw[a] / d;
        out[a] = v;
        den += v;
    }
    if (hit >= 0) {
        for (int a = 0; a < p; ++a) out[a] = (a == hit) ? T(1) : T(0);
        return;
    }
    T inv = T(1) / den;
    for (int a = 0; a < p; ++a) out[a] *= inv;
}

__device__ inline double box_side(int level) { return ldexp(1.0, -level); }

// ------------------------------------------------------------------ upward
// acc[a0][a1] over the p^2 outputs; thread t owns outputs t, t + TPB, ...
template <int P>
constexpr int nown() { return (P * P + TPB - 1) / TPB; }

// COH: the box's F_out children were computed by the same launch (queue-fed)
template <typename T, int P, bool COH>
__device__ __forceinline__ void upward2_box(const Dev2<T> &D, const int32_t B)
{
    constexpr int P2 = P * P, NO = nown<P>(), CH = 64;
    __shared__ T Am[2 * P2], xc[P], bw[P], tmp[P2], cs[P2], L0[CH * P], L1[CH * P], qq[CH];
    for (int t = threadIdx.x; t < 2 * P2; t += TPB) Am[t] = D.c2p[t];
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    T acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = T(0);
    const double cx = D.bcenter[2 * (int64_t)B], cy = D.bcenter[2 * (int64_t)B + 1];
    const double sc = 2.0 / box_side(D.blevel[B]);
    __syncthreads();
    for (int k = 0; k < 4; ++k) {
        const int32_t C = D.child0[B] + k;
        const int cnt = D.pcount[C];
        if (cnt == 0) continue;
        if (D.bflags[C] & 2) {
            const T *Ax = Am + ((k >> 1) & 1) * P2, *Ay = Am + (k & 1) * P2;
            __syncthreads();
            copy_to_lds<COH, TPB>(cs, D.proxy + (int64_t)D.proxy_slot[C] * P2, P2);
            __syncthreads();
            // tmp[i0][a1] = sum_i1 cs[i0][i1] Ay[a1][i1]
            for (int t = threadIdx.x; t < P2; t += TPB) {
                const int i0 = t / P, a1 = t % P;
                T s = T(0);
                for (int i1 = 0; i1 < P; ++i1) s += cs[i0 * P + i1] * Ay[a1 * P + i1];
                tmp[t] = s;
            }
            __syncthreads();
            // acc[a0][a1] += sum_i0 Ax[a0][i0] tmp[i0][a1]
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const int t = threadIdx.x + o * TPB;
                if (t < P2) {
                    const int a0 = t / P, a1 = t % P;
                    T s = T(0);
                    for (int i0 = 0; i0 < P; ++i0) s += Ax[a0 * P + i0] * tmp[i0 * P + a1];
                    acc[o] += s;
                }
            }
        } else {
            const int64_t i0 = D.pstart[C];
            for (int base = 0; base < cnt; base += CH) {
                const int m = min(CH, cnt - base);
                __syncthreads();
                for (int t = threadIdx.x; t < 2 * m; t += TPB) {
                    const int pt = t / 2, d = t % 2;
                    const int64_t i = i0 + base + pt;
                    const double x = (d == 0) ? (D.X[i] - cx) * sc : (D.Y[i] - cy) * sc;
                    lagrange_row<T>(P, xc, bw, (T)x, (d == 0 ? L0 : L1) + pt * P);
                }
                for (int t = threadIdx.x; t < m; t += TPB) qq[t] = (T)D.qs[i0 + base + t];
                __syncthreads();
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    const int t = threadIdx.x + o * TPB;
                    if (t < P2) {
                        const int a0 = t / P, a1 = t % P;
                        T s = T(0);
                        for (int pt = 0; pt < m; ++pt) s += L0[pt * P + a0] * L1[pt * P + a1] * qq[pt];
                        acc[o] += s;
                    }
                }
            }
        }
    }
    T *dst = D.proxy + (int64_t)D.proxy_slot[B] * P2;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const int t = threadIdx.x + o * TPB;
        if (t < P2) st_c<COH>(dst + t, acc[o]);
    }
}

// one level's F_out boxes, one workgroup per box
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_upward2(Dev2<T> D, const int32_t *list)
{
    upward2_box<T, P, false>(D, list[blockIdx.x]);
}

// the F_out boxes of every level, finest first, from the work queue (a box
// waits for its F_out children)
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_upward2_q(Dev2<T> D, WorkQ q)
{
    queue_loop(
        q,
        [&](int32_t B) {
            if (threadIdx.x < 4) {
                const int32_t C = D.child0[B] + threadIdx.x;
                if (D.pcount[C] > 0 && (D.bflags[C] & 2)) wait_done(q, C);
            }
        },
        [&](int32_t B) { upward2_box<T, P, true>(D, B); });
}

// --------------------------------------------------------------- root W_0
// One block per problem, FP64: proxies of the root (its F_out proxies, or
// its points anterpolated), plane waves of spacing hw, weights, values on
// the root grid, plus C_b times the total charge.
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_root2(Dev2<T> D, int npmax)
{
    constexpr int P2 = P * P;
    extern __shared__ __align__(16) double rsm[];
    const int nwn = D.nwn, nwh = D.nwh, nw = D.nw;
    double *rho = rsm;                    // p^2
    double *t1r = rho + P2, *t1i = t1r + P * nwh;         // [j1][m2]
    double *fr = t1i + P * nwh, *fi = fr + nwn * nwh;     // [m1][m2]
    double *g1r = fi + nwn * nwh, *g1i = g1r + P * nwh;   // [j1][m2]
    double *xc = g1i + P * nwh, *bw = xc + P;
    double *L = bw + P;                                   // [npmax][2][P]
    __shared__ double red[TPB];
    const int b = blockIdx.x;
    const int32_t R = b;  // level-0 box b is the root of problem b
    const int cnt = D.pcount[R];
    if (cnt == 0) return;  // whole block
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb64[t]; bw[t] = D.bary64[t]; }
    // total charge of the problem
    double qsum = 0.0;
    for (int i = threadIdx.x; i < cnt; i += TPB) qsum += D.qs[D.pstart[R] + i];
    red[threadIdx.x] = qsum;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double Q = red[0];
    if (D.bflags[R] & 2) {
        const T *src = D.proxy + (int64_t)D.proxy_slot[R] * P2;
        for (int t = threadIdx.x; t < P2; t += TPB) rho[t] = (double)src[t];
    } else {
        // a root leaf holds at most npmax points
        const int64_t i0 = D.pstart[R];
        for (int t = threadIdx.x; t < 2 * cnt; t += TPB) {
            const int pt = t / 2, d = t % 2;
            const double x = (d == 0 ? D.X[i0 + pt] : D.Y[i0 + pt]) * 2.0;  // root centre 0, side 1
            lagrange_row<double>(P, xc, bw, x, L + (pt * 2 + d) * P);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < P2; t += TPB) {
            const int a0 = t / P, a1 = t % P;
            double s = 0.0;
            for (int pt = 0; pt < cnt; ++pt) s += L[(pt * 2) * P + a0] * L[(pt * 2 + 1) * P + a1] * D.qs[i0 + pt];
            rho[t] = s;
        }
    }
    __syncthreads();
    // E_W[m][j] = exp(-i hw m x_j / 2): ew64[((m + nw) P + j) 2 + {0,1}]
    // t1[j1][m2] = sum_j2 rho[j1][j2] E_W[m2][j2], m2 >= 0
    for (int t = threadIdx.x; t < P * nwh; t += TPB) {
        const int j1 = t / nwh, m2 = t % nwh;
        double sr = 0.0, si = 0.0;
        for (int j2 = 0; j2 < P; ++j2) {
            const double *e = D.ew64 + ((int64_t)(m2 + nw) * P + j2) * 2;
            sr += rho[j1 * P + j2] * e[0];
            si += rho[j1 * P + j2] * e[1];
        }
        t1r[t] = sr;
        t1i[t] = si;
    }
    __syncthreads();
    // F[m1][m2] = w(m) sum_j1 E_W[m1][j1] t1[j1][m2]
    for (int t = threadIdx.x; t < nwn * nwh; t += TPB) {
        const int m1 = t / nwh, m2 = t % nwh;
        double sr = 0.0, si = 0.0;
        for (int j1 = 0; j1 < P; ++j1) {
            const double *e = D.ew64 + ((int64_t)m1 * P + j1) * 2;
            const double ar = t1r[j1 * nwh + m2], ai = t1i[j1 * nwh + m2];
            sr += e[0] * ar - e[1] * ai;
            si += e[0] * ai + e[1] * ar;
        }
        const double w = D.kern ? D.yww[(int64_t)b * nwn * nwh + t] : D.ww64[t];
        fr[t] = sr * w;
        fi[t] = si * w;
    }
    __syncthreads();
    // g[j1][m2] = sum_m1 conj(E_W[m1][j1]) F[m1][m2]
    for (int t = threadIdx.x; t < P * nwh; t += TPB) {
        const int j1 = t / nwh, m2 = t % nwh;
        double sr = 0.0, si = 0.0;
        for (int m1 = 0; m1 < nwn; ++m1) {
            const double *e = D.ew64 + ((int64_t)m1 * P + j1) * 2;
            const double ar = fr[m1 * nwh + m2], ai = fi[m1 * nwh + m2];
            sr += e[0] * ar + e[1] * ai;
            si += e[0] * ai - e[1] * ar;
        }
        g1r[t] = sr;
        g1i[t] = si;
    }
    __syncthreads();
    // v[j1][j2] = sum_m2 c_m2 Re(conj(E_W[m2][j2]) g[j1][m2]) + C_b Q
    const double Cb = D.kern ? 0.0 : -log(D.pside[b]) / (2.0 * M_PI);
    for (int t = threadIdx.x; t < P2; t += TPB) {
        const int j1 = t / P, j2 = t % P;
        double s = 0.0;
        for (int m2 = 0; m2 < nwh; ++m2) {
            const double *e = D.ew64 + ((int64_t)(m2 + nw) * P + j2) * 2;
            const double v = e[0] * g1r[j1 * nwh + m2] + e[1] * g1i[j1 * nwh + m2];
            s += (m2 == 0) ? v : 2.0 * v;
        }
        D.w0vals[(int64_t)b * P2 + t] = (T)(s + Cb * Q);
    }
}

// -------------------------------------------- proxies -> plane waves
// Phi[m1][m2] = sum_j E[m1][j1] E[m2][j2] rho[j1][j2], E[m][j] = exp(-i pi m x_j/3), m2 >= 0
template <typename T, int P, int NF>
__global__ void __launch_bounds__(TPB) k_proxy2pw2(Dev2<T> D, const int32_t *list)
{
    constexpr int P2 = P * P, NN = 2 * NF + 1, NH = NF + 1;
    __shared__ T rho[P2], Er[NN * P], Ei[NN * P], tr[P * NH], ti[P * NH];
    const int32_t B = list[blockIdx.x];
    const T *src = D.proxy + (int64_t)D.proxy_slot[B] * P2;
    for (int t = threadIdx.x; t < P2; t += TPB) rho[t] = src[t];
    for (int t = threadIdx.x; t < NN * P; t += TPB) {
        Er[t] = D.epw[2 * t];
        Ei[t] = D.epw[2 * t + 1];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P * NH; t += TPB) {
        const int j1 = t / NH, m2 = t % NH;
        T sr = T(0), si = T(0);
        for (int j2 = 0; j2 < P; ++j2) {
            const T r = rho[j1 * P + j2];
            sr += r * Er[(m2 + NF) * P + j2];
            si += r * Ei[(m2 + NF) * P + j2];
        }
        tr[t] = sr;
        ti[t] = si;
    }
    __syncthreads();
    const int64_t nm = D.pwstride;
    T *outr = D.phi + 2 * (int64_t)D.proxy_slot[B] * nm, *outi = outr + nm;
    for (int t = threadIdx.x; t < NN * NH; t += TPB) {
        const int m1 = t / NH, m2 = t % NH;
        T sr = T(0), si = T(0);
        for (int j1 = 0; j1 < P; ++j1) {
            const T er = Er[m1 * P + j1], ei = Ei[m1 * P + j1];
            const T ar = tr[j1 * NH + m2], ai = ti[j1 * NH + m2];
            sr += er * ar - ei * ai;
            si += er * ai + ei * ar;
        }
        outr[t] = sr;
        outi[t] = si;
    }
}

// ------------------------------------------------ diagonal translation
// Children t = (x y bits) of one parent at cells t + (1,1) of the 4x4 block
// of boxes around them; with delta = (c_S - c_B)/s_l the factor is
// w^{-(m.delta)}, w = e^{2 pi i/3}, separable: a y pass then an x pass.
template <typename T>
struct Cx2 { T r, i; };

template <typename T>
__device__ inline Cx2<T> cmul2(Cx2<T> a, Cx2<T> f) { return {a.r * f.r - a.i * f.i, a.r * f.i + a.i * f.r}; }

template <typename T>
__device__ inline Cx2<T> root3b(int k)  // w^{-k}
{
    k %= 3;
    if (k < 0) k += 3;
    const T s3 = T(0.86602540378443864676);
    if (k == 0) return {T(1), T(0)};
    if (k == 1) return {T(-0.5), -s3};
    return {T(-0.5), s3};
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_pwshift2(Dev2<T> D, const int32_t *oct_dst, const int32_t *oct_src,
                                                  const int32_t *oct_level, const int32_t *oct_prob, int64_t noct,
                                                  int nchunk)
{
    __shared__ int32_t src[16];
    __shared__ int32_t dst[4];
    const int64_t G = gridDim.x;  // a multiple of 8
    const int64_t Lb = (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8;
    const int64_t o = Lb / nchunk;
    const int chunk = (int)(Lb % nchunk);
    if (o >= noct) return;  // whole block: before any barrier
    if (threadIdx.x < 16) src[threadIdx.x] = oct_src[o * 16 + threadIdx.x];
    if (threadIdx.x < 4) dst[threadIdx.x] = oct_dst[o * 4 + threadIdx.x];
    __syncthreads();
    const int64_t nm = D.pwstride;
    const int64_t e = (int64_t)chunk * TPB + threadIdx.x;
    if (e >= nm) return;
    const int nh = D.nh, nf = D.nf;
    const int m1 = (int)(e / nh) - nf, m2 = (int)(e % nh);
    const Cx2<T> xm = root3b<T>(-m1), xp = root3b<T>(m1), ym = root3b<T>(-m2), yp = root3b<T>(m2);
    const Cx2<T> one = {T(1), T(0)};
    Cx2<T> acc[2][2] = {{{T(0), T(0)}, {T(0), T(0)}}, {{T(0), T(0)}, {T(0), T(0)}}};
    const T *phi = D.phi;
#pragma unroll
    for (int gx = 0; gx < 4; ++gx) {
        Cx2<T> f[4];
        bool any = false;
#pragma unroll
        for (int gy = 0; gy < 4; ++gy) {
            const int32_t sl = src[gx * 4 + gy];
            if (sl >= 0) {
                const T *q = phi + 2 * (int64_t)sl * nm + e;
                f[gy] = {q[0], q[nm]};
                any = true;
            } else {
                f[gy] = {T(0), T(0)};
            }
        }
        if (!any) continue;
        // Y[ty] = sum over gy = ty .. ty+2 of w^{-m2 (gy - ty - 1)} f[gy]
        Cx2<T> y0 = cmul2(f[0], ym), y1 = cmul2(f[3], yp);
        const Cx2<T> a2 = cmul2(f[2], yp), a1 = cmul2(f[1], ym);
        y0.r += f[1].r + a2.r; y0.i += f[1].i + a2.i;
        y1.r += f[2].r + a1.r; y1.i += f[2].i + a1.i;
        if (gx <= 2) {
            const Cx2<T> fx = (gx == 0) ? xm : (gx == 1) ? one : xp;
            const Cx2<T> v0 = cmul2(y0, fx), v1 = cmul2(y1, fx);
            acc[0][0].r += v0.r; acc[0][0].i += v0.i;
            acc[0][1].r += v1.r; acc[0][1].i += v1.i;
        }
        if (gx >= 1) {
            const Cx2<T> fx = (gx == 1) ? xm : (gx == 2) ? one : xp;
            const Cx2<T> v0 = cmul2(y0, fx), v1 = cmul2(y1, fx);
            acc[1][0].r += v0.r; acc[1][0].i += v0.i;
            acc[1][1].r += v1.r; acc[1][1].i += v1.i;
        }
    }
    // the log kernel's weights are the same at every level; K_0's depend on
    // the problem and the level
    const T w = D.kern ? D.ywd[((int64_t)oct_prob[o] * D.nlev + oct_level[o]) * nm + e] : D.wd0[e];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int32_t d = dst[t];
        if (d < 0) continue;
        const Cx2<T> v = acc[t >> 1][t & 1];
        T *out = D.psi + 2 * (int64_t)d * nm + e;
        out[0] = v.r * w;
        out[nm] = v.i * w;
    }
}

// ------------------------------------------------ local values (anchors)
// COH: the anchor above the box was computed by the same launch (queue-fed)
template <typename T, int P, int NF, bool COH>
__device__ __forceinline__ void local2_box(const Dev2<T> &D, const int32_t B, const int level)
{
    constexpr int P2 = P * P, NN = 2 * NF + 1, NH = NF + 1, NO = nown<P>();
    __shared__ T Er[NN * P], Ei[NN * P], xc[P], bw[P], v[P2], tmp[P2], Mx[P2], My[P2];
    __shared__ T gr[P * NH], gi[P * NH];
    for (int t = threadIdx.x; t < NN * P; t += TPB) {
        Er[t] = D.epw[2 * t];
        Ei[t] = D.epw[2 * t + 1];
    }
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    T acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = T(0);
    __syncthreads();
    if (level == 0) {
        const T *w0 = D.w0vals + (int64_t)D.bprob[B] * P2;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int t = threadIdx.x + o * TPB;
            if (t < P2) acc[o] = w0[t];
        }
    } else {
        // node i of B sits at A-coordinate ((c_B + s_B x_i / 2) - c_A) * 2 / s_A
        const int32_t A = D.anchor[D.parent[B]];
        const double sB = box_side(level), sA = box_side(D.blevel[A]);
        for (int t = threadIdx.x; t < 2 * P; t += TPB) {
            const int d = t / P, i = t % P;
            const double xi =
                (D.bcenter[2 * (int64_t)B + d] + 0.5 * sB * D.xcheb64[i] - D.bcenter[2 * (int64_t)A + d]) * (2.0 / sA);
            lagrange_row<T>(P, xc, bw, (T)xi, (d == 0 ? Mx : My) + i * P);
        }
        copy_to_lds<COH, TPB>(v, D.local + (int64_t)D.local_slot[A] * P2, P2);
        __syncthreads();
        // tmp[a0][i1] = sum_a1 v[a0][a1] My[i1][a1]
        for (int t = threadIdx.x; t < P2; t += TPB) {
            const int a0 = t / P, i1 = t % P;
            T s = T(0);
            for (int a1 = 0; a1 < P; ++a1) s += v[a0 * P + a1] * My[i1 * P + a1];
            tmp[t] = s;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int t = threadIdx.x + o * TPB;
            if (t < P2) {
                const int i0 = t / P, i1 = t % P;
                T s = T(0);
                for (int a0 = 0; a0 < P; ++a0) s += Mx[i0 * P + a0] * tmp[a0 * P + i1];
                acc[o] = s;
            }
        }
    }
    if (D.psi_slot[B] >= 0) {
        const int64_t nm = D.pwstride;
        const T *psr = D.psi + 2 * (int64_t)D.psi_slot[B] * nm, *psi = psr + nm;
        __syncthreads();
        // g[j1][m2] = sum_m1 conj(E[m1][j1]) Psi[m1][m2]
        for (int t = threadIdx.x; t < P * NH; t += TPB) {
            const int j1 = t / NH, m2 = t % NH;
            T sr = T(0), si = T(0);
            for (int m1 = 0; m1 < NN; ++m1) {
                const T er = Er[m1 * P + j1], ei = Ei[m1 * P + j1];
                const T ar = psr[m1 * NH + m2], ai = psi[m1 * NH + m2];
                sr += er * ar + ei * ai;
                si += er * ai - ei * ar;
            }
            gr[t] = sr;
            gi[t] = si;
        }
        __syncthreads();
        // acc[j1][j2] += sum_m2 c_m2 Re(conj(E[m2][j2]) g[j1][m2])
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int t = threadIdx.x + o * TPB;
            if (t < P2) {
                const int j1 = t / P, j2 = t % P;
                T s = T(0);
                for (int m2 = 0; m2 < NH; ++m2) {
                    const T val = Er[(m2 + NF) * P + j2] * gr[j1 * NH + m2] + Ei[(m2 + NF) * P + j2] * gi[j1 * NH + m2];
                    s += (m2 == 0) ? val : T(2) * val;
                }
                acc[o] += s;
            }
        }
    }
    // a finer anchor of the same launch reads these values: past the caches
    T *dst = D.local + (int64_t)D.local_slot[B] * P2;
    if (COH && D.anc_read[D.local_slot[B]]) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int t = threadIdx.x + o * TPB;
            if (t < P2) st_c<true>(dst + t, acc[o]);
        }
    } else {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int t = threadIdx.x + o * TPB;
            if (t < P2) dst[t] = acc[o];
        }
    }
}

// one level's anchors, one workgroup per box
template <typename T, int P, int NF>
__global__ void __launch_bounds__(TPB) k_local_pw2(Dev2<T> D, const int32_t *list, int level)
{
    local2_box<T, P, NF, false>(D, list[blockIdx.x], level);
}

// the anchors of every level, coarsest first, from the work queue (a box
// below a root waits for the anchor of its parent); one box per workgroup
// (a box loop held more registers and halved the occupancy)
template <typename T, int P, int NF>
__global__ void __launch_bounds__(TPB) k_local_pw2_q(Dev2<T> D, WorkQ q)
{
    queue_item(
        q,
        [&](int32_t B) {
            if (threadIdx.x == 0 && D.blevel[B] > 0) wait_done(q, D.anchor[D.parent[B]]);
        },
        [&](int32_t B) { local2_box<T, P, NF, true>(D, B, D.blevel[B]); });
}

// ------------------------------------------------------------ leaf targets
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_leaf2(Dev2<T> D, const int32_t *anc, const int32_t *tbeg, const int32_t *tgt)
{
    constexpr int P2 = P * P;
    __shared__ T v[P2], xc[P], bw[P];
    const int a = blockIdx.x;
    const int b0 = tbeg[a], b1 = tbeg[a + 1];
    if (b0 == b1) return;
    const int32_t A = anc[a];
    const T *src = D.local + (int64_t)a * P2;
    for (int t = threadIdx.x; t < P2; t += TPB) v[t] = src[t];
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    __syncthreads();
    const double cA0 = D.bcenter[2 * (int64_t)A], cA1 = D.bcenter[2 * (int64_t)A + 1];
    const double sc = 2.0 / box_side(D.blevel[A]);
    for (int t = b0 + threadIdx.x; t < b1; t += TPB) {
        const int64_t i = tgt[t];
        T lx[P], ly[P];
        lagrange_row_fast<T, P>(xc, bw, (T)((D.X[i] - cA0) * sc), lx);
        lagrange_row_fast<T, P>(xc, bw, (T)((D.Y[i] - cA1) * sc), ly);
        T u = T(0);
        for (int j1 = 0; j1 < P; ++j1) {
            T s = T(0);
#pragma unroll
            for (int j2 = 0; j2 < P; ++j2) s += v[j1 * P + j2] * ly[j2];
            u += lx[j1] * s;
        }
        D.ufar[i] = (double)u;
    }
}

// -------------------------------------------------------- residual sums
// For a source in terminal box T at level l and r < s_l:
//   R_l(r) = -log(r^2)/(4 pi) - l log(2)/(2 pi) - m(r/s_l)
// and at r = 0 the far field's own share is removed:
//   -(m(0) + l log(2)/(2 pi) + C_b) times the charge.
// The residual's source staging, shared by the two kernels below.  The
// running source counts of a leaf's gather list and the entries' first points
// and levels sit in dynamic LDS (loff: L + 1 entries, then lbeg, llev: L each;
// sized at launch to the plan's longest list), so that staging a source is one
// dependent global load.  Only the sources that can reach the bounding box of
// the chunk's targets are staged: the residual vanishes beyond the source box
// side s, and a source farther than s from the box is farther than s from
// every target (the box distance is formed with the same rounded operations
// as the pair distances, so it is not larger than any pair's; the margin keeps
// the comparison safe).

// bounding box of the chunk's targets (wave 0 holds them all: tch <= 64):
// bb = {xlo, ylo, xhi, yhi}
template <typename T>
__device__ __forceinline__ void target_box2(T xt, T yt, T *bb)
{
    if ((threadIdx.x >> 6) != 0) return;
    T b[4] = {xt, yt, -xt, -yt};
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = min(b[k], __shfl_xor(b[k], d));
    if ((threadIdx.x & 63) == 0) {
        bb[0] = b[0];
        bb[1] = b[1];
        bb[2] = -b[2];
        bb[3] = -b[3];
    }
}

// stage the next sources of the list, from `cursor` on, that can reach the box
// (rounds of TPB entries while a whole round still fits); returns how many
template <typename T, int RCAP>
__device__ __forceinline__ int stage_sources2(const Dev2<T> &D, const int32_t *loff, const int32_t *lbeg,
                                              const int32_t *llev, int L, int nsrc, int &cursor, double cx, double cy,
                                              const T *bb, int *wtot, T *sx, T *sy, T *sq, T *sis2, T *slc)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cnt = 0;
    __syncthreads();
    while (cursor < nsrc && cnt <= RCAP - TPB) {
        const int g = cursor + threadIdx.x;
        bool keep = false;
        T ux = T(0), uy = T(0), uq = T(0), uis2 = T(0), ulc = T(0);
        if (g < nsrc) {
            int lo = 0, hi = L - 1;  // entry k with loff[k] <= g < loff[k+1]
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (loff[mid] <= g) lo = mid; else hi = mid - 1;
            }
            const int64_t j = (int64_t)lbeg[lo] + (g - loff[lo]);
            const int lev = llev[lo];
            ux = (T)(D.X[j] - cx);
            uy = (T)(D.Y[j] - cy);
            uq = (T)D.qs[j];
            uis2 = (T)ldexp(1.0, 2 * lev);
            ulc = D.kern ? (T)lev : (T)(-lev * M_LN2 / (2.0 * M_PI));
            const T ex = max(max(bb[0] - ux, T(0)), ux - bb[2]);
            const T ey = max(max(bb[1] - uy, T(0)), uy - bb[3]);
            const T d2 = ex * ex + ey * ey;
            keep = d2 * uis2 < T(1.0001);
        }
        const uint64_t m = __ballot(keep);
        if (lane == 0) wtot[wv] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < TPB / 64; ++k) {
            const int c = wtot[k];
            before += k < wv ? c : 0;
            total += c;
        }
        if (keep) {
            const int pos = cnt + before + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            sx[pos] = ux;
            sy[pos] = uy;
            sq[pos] = uq;
            sis2[pos] = uis2;
            slc[pos] = ulc;
        }
        cnt += total;
        cursor += TPB;
        __syncthreads();
    }
    return cnt;
}

// the list's running counts, first points and levels into dynamic LDS
template <typename T>
__device__ __forceinline__ void load_list2(const Dev2<T> &D, const int32_t *nl_src, const int32_t *nl_pre, int32_t l0,
                                           int L, int32_t *loff, int32_t *lbeg, int32_t *llev)
{
    for (int k = threadIdx.x; k <= L; k += TPB) loff[k] = nl_pre[l0 + blockIdx.x + k];
    for (int k = threadIdx.x; k < L; k += TPB) {
        const int32_t Tb = nl_src[l0 + k];
        lbeg[k] = D.pstart[Tb];
        llev[k] = D.blevel[Tb];
    }
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_residual2(Dev2<T> D, const int32_t *leaves, const int32_t *nl_off,
                                                   const int32_t *nl_src, const int32_t *nl_pre)
{
    constexpr int RCAP = sizeof(T) == 8 ? 768 : 1024;
    constexpr int YLEV = 32;  // levels of a K_0 problem's tables held in LDS
    __shared__ T sx[RCAP], sy[RCAP], sq[RCAP], sis2[RCAP], slc[RCAP];
    extern __shared__ __align__(16) int32_t loff[];  // then lbeg, llev (load_list2)
    __shared__ int wtot[TPB / 64];
    __shared__ T tbb[4];
    __shared__ T gc[48];
    __shared__ T yc[YLEV * 48];
    __shared__ T yself[YLEV];
    __shared__ double part[TPB];
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = D.pstart[B];
    const int nt = D.pcount[B];
    const int32_t l0 = nl_off[blockIdx.x];
    const int L = nl_off[blockIdx.x + 1] - l0;
    const int deg = D.kern ? D.ydeg : D.gdeg;
    const int32_t prob = D.bprob[B];
    if (D.kern) {
        for (int t = threadIdx.x; t < D.nlev * 48; t += TPB) yc[t] = D.ycheb[(int64_t)prob * D.nlev * 48 + t];
        for (int t = threadIdx.x; t < D.nlev; t += TPB) yself[t] = (T)D.yself[(int64_t)prob * D.nlev + t];
    } else {
        for (int t = threadIdx.x; t <= deg; t += TPB) gc[t] = D.gcheb[t];
    }
    int32_t *lbeg = loff + L + 1, *llev = lbeg + L;
    load_list2(D, nl_src, nl_pre, l0, L, loff, lbeg, llev);
    __syncthreads();
    const int nsrc = loff[L];
    const double cx = D.bcenter[2 * (int64_t)B], cy = D.bcenter[2 * (int64_t)B + 1];
    const double Cb = D.kern ? 0.0 : -log(D.pside[prob]) / (2.0 * M_PI);
    const T lam = D.kern ? (T)D.ylam[prob] : T(0);
    const T zero_val = (T)(-(D.m0 + Cb));  // plus slc of the source level
    const T k4pi = (T)(-1.0 / (4.0 * M_PI));
    // one thread per target and source share; a leaf of nt <= 64 targets uses
    // TPB/nt shares so that few threads idle
    const int tch = min(max(nt, 1), 64);
    const int nsplit = TPB / tch;
    const int tl = threadIdx.x % tch, split = threadIdx.x / tch;
    for (int tbase = 0; tbase < nt; tbase += tch) {
        const bool active = (tbase + tl) < nt;
        const int64_t it = t0 + tbase + (active ? tl : 0);
        const T xt = (T)(D.X[it] - cx), yt = (T)(D.Y[it] - cy);
        target_box2(xt, yt, tbb);
        double acc = 0.0;
        for (int cursor = 0; cursor < nsrc;) {
            const int cnt =
                stage_sources2<T, RCAP>(D, loff, lbeg, llev, L, nsrc, cursor, cx, cy, tbb, wtot, sx, sy, sq, sis2, slc);
            T pacc = T(0);
            if (D.kern) {
                // K_0(lambda r) - M_l(r) for 0 < r < s_l; -M_l(0) at r = 0
                for (int j = split; j < cnt && split < nsplit; j += nsplit) {
                    const T dx = xt - sx[j], dy = yt - sy[j];
                    const T r2 = dx * dx + dy * dy;
                    const T tt = r2 * sis2[j];
                    if (tt < T(1)) {
                        const int lv = (int)slc[j];
                        T val;
                        if (r2 > T(0)) {
                            const T *cf = yc + lv * 48;
                            const T u = T(2) * tt - T(1);
                            T b1 = T(0), b2 = T(0);
                            for (int k = deg; k >= 1; --k) {
                                T b0 = cf[k] + T(2) * u * b1 - b2;
                                b2 = b1;
                                b1 = b0;
                            }
                            val = bessel_k0<T>(lam * sqrt(r2)) - (cf[0] + u * b1 - b2);
                        } else {
                            val = -yself[lv];
                        }
                        pacc += sq[j] * val;
                    }
                }
                acc += (double)pacc;
                continue;
            }
            for (int j = split; j < cnt && split < nsplit; j += nsplit) {
                const T dx = xt - sx[j], dy = yt - sy[j];
                const T r2 = dx * dx + dy * dy;
                const T tt = r2 * sis2[j];
                if (tt < T(1)) {
                    T val;
                    if (r2 > T(0)) {
                        const T u = T(2) * tt - T(1);
                        T b1 = T(0), b2 = T(0);
                        for (int k = deg; k >= 1; --k) {
                            T b0 = gc[k] + T(2) * u * b1 - b2;
                            b2 = b1;
                            b1 = b0;
                        }
                        val = k4pi * log(r2) - (gc[0] + u * b1 - b2);
                    } else {
                        val = zero_val;
                    }
                    pacc += sq[j] * (val + slc[j]);
                }
            }
            acc += (double)pacc;
        }
        __syncthreads();
        part[threadIdx.x] = acc;
        __syncthreads();
        if (split == 0 && active) {
            double sum = 0.0;
            for (int k = 0; k < nsplit; ++k) sum += part[k * tch + tl];
            D.ures[t0 + tbase + tl] = sum;
        }
    }
}

// log(x) for x > 0: the hardware base-2 logarithm in FP32 (operands below
// 1e-30, never produced by distinct points of a normalised tree, go through
// the library function), the library function in FP64
__device__ inline float log_r2(float x) { return x > 1e-30f ? 0.69314718055994531f * __builtin_amdgcn_logf(x) : logf(x); }
__device__ inline double log_r2(double x) { return log(x); }

// Residual sums of -log(r)/(2 pi) in gather form, the same layout as
// k_residual2 (which keeps the K_0 kernel): per pair with x = r/s_l < 1,
//   -log(r^2)/(4 pi) - m(x) + level constant,
// m as a power series of degree DEG in u = 2x^2 - 1 held in registers and
// evaluated by Horner's rule; RB candidates per round are read and tested
// together, then the ones in range are summed.
template <typename T, int DEG>
__global__ void __launch_bounds__(TPB) k_residual2_log(Dev2<T> D, const int32_t *leaves, const int32_t *nl_off,
                                                       const int32_t *nl_src, const int32_t *nl_pre)
{
    constexpr int RCAP = 512;
    __shared__ union {
        struct { T x[RCAP], y[RCAP], q[RCAP], is2[RCAP], lc[RCAP]; } s;
        double part[TPB];
    } stg;
    T *sx = stg.s.x, *sy = stg.s.y, *sq = stg.s.q, *sis2 = stg.s.is2, *slc = stg.s.lc;
    double *part = stg.part;
    extern __shared__ __align__(16) int32_t loff[];  // then lbeg, llev (load_list2)
    __shared__ int wtot[TPB / 64];
    __shared__ T tbb[4];
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = D.pstart[B];
    const int nt = D.pcount[B];
    const int32_t l0 = nl_off[blockIdx.x];
    const int L = nl_off[blockIdx.x + 1] - l0;
    T gm[DEG + 1];
#pragma unroll
    for (int k = 0; k <= DEG; ++k) gm[k] = (k <= D.gdeg) ? D.gmono[k] : T(0);
    int32_t *lbeg = loff + L + 1, *llev = lbeg + L;
    load_list2(D, nl_src, nl_pre, l0, L, loff, lbeg, llev);
    __syncthreads();
    const int nsrc = loff[L];
    const int32_t prob = D.bprob[B];
    const double cx = D.bcenter[2 * (int64_t)B], cy = D.bcenter[2 * (int64_t)B + 1];
    const double Cb = -log(D.pside[prob]) / (2.0 * M_PI);
    const T zero_val = (T)(-(D.m0 + Cb));  // plus the source level's constant
    const T k4pi = (T)(-1.0 / (4.0 * M_PI));
    const int tch = min(max(nt, 1), 64);
    const int nsplit = TPB / tch;
    const int tl = threadIdx.x % tch, split = threadIdx.x / tch;
    for (int tbase = 0; tbase < nt; tbase += tch) {
        const bool active = (tbase + tl) < nt;
        const int64_t it = t0 + tbase + (active ? tl : 0);
        const T xt = (T)(D.X[it] - cx), yt = (T)(D.Y[it] - cy);
        target_box2(xt, yt, tbb);
        double acc = 0.0;
        for (int cursor = 0; cursor < nsrc;) {
            const int cnt =
                stage_sources2<T, RCAP>(D, loff, lbeg, llev, L, nsrc, cursor, cx, cy, tbb, wtot, sx, sy, sq, sis2, slc);
            T pacc = T(0);
            constexpr int RB = 4;
            for (int j0 = split; j0 < cnt && split < nsplit; j0 += RB * nsplit) {
                T r2v[RB], ttv[RB];
                int jv[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int j = j0 + u * nsplit;
                    jv[u] = j < cnt ? j : -1;
                    const int jj = j < cnt ? j : j0;  // a valid slot for the spare lanes
                    const T dx = xt - sx[jj], dy = yt - sy[jj];
                    r2v[u] = dx * dx + dy * dy;
                    ttv[u] = r2v[u] * sis2[jj];
                }
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    if (jv[u] >= 0 && ttv[u] < T(1)) {
                        const int j = jv[u];
                        const T uu = T(2) * ttv[u] - T(1);
                        T m = gm[DEG];
#pragma unroll
                        for (int k = DEG - 1; k >= 0; --k) m = m * uu + gm[k];
                        const T val = (r2v[u] > T(0)) ? k4pi * log_r2(r2v[u]) - m : zero_val;
                        pacc += sq[j] * (val + slc[j]);
                    }
                }
            }
            acc += (double)pacc;
        }
        __syncthreads();
        part[threadIdx.x] = acc;
        __syncthreads();
        if (split == 0 && active) {
            double sum = 0.0;
            for (int k = 0; k < nsplit; ++k) sum += part[k * tch + tl];
            D.ures[t0 + tbase + tl] = sum;
        }
    }
}

// the residual launch: K_0 problems in k_residual2, the log kernel in
// k_residual2_log with the series' degree as a compile-time bucket
template <typename T>
static void launch_residual2(const Dev2<T> &D, Plan *Pl, hipStream_t s)
{
    const dim3 g((unsigned)Pl->nleaf), b(TPB);
    const size_t lds = sizeof(int32_t) * 3 * ((size_t)Pl->nl_max + 1);  // loff, lbeg, llev
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    };
    if (D.kern) go(k_residual2<T>);
    else if (D.gdeg <= 9) go(k_residual2_log<T, 9>);
    else if (D.gdeg <= 13) go(k_residual2_log<T, 13>);
    else if (D.gdeg <= 17) go(k_residual2_log<T, 17>);
    else if (D.gdeg <= 23) go(k_residual2_log<T, 23>);
    else go(k_residual2_log<T, 47>);
}

__global__ void k_gather_q2(const double *charges, const int32_t *perm, int64_t n, double *qs)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) qs[i] = charges[perm[i]];
}

__global__ void k_finalize2(const double *ufar, const double *ures, const int32_t *perm, int64_t n, double *pot,
                            double *farp, double *nearp)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    double f = ufar[i], r = ures[i];
    if (pot) pot[j] = f + r;
    if (farp) farp[j] = f;
    if (nearp) nearp[j] = r;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

template <typename T>
Dev2<T> make_dev2(Plan *P)
{
    Dev2<T> D;
    const Tables &t = P->tab;
    D.p = t.p; D.nf = t.nf; D.nn = t.nn; D.nh = t.nh; D.nw = t.nw; D.nwn = t.nwn; D.nwh = t.nwh;
    D.gdeg = sizeof(T) == 8 ? t.gdeg : t.gdeg32;
    D.nprob = P->nprob;
    D.m0 = t.m0;
    D.kern = (P->kernel == DMK_YUKAWA) ? 1 : 0;
    D.nlev = P->nlevels;
    D.ydeg = sizeof(T) == 8 ? P->y_deg : P->y_deg32;
    D.ywd = (const T *)(sizeof(T) == 8 ? (void *)P->y_wd64 : (void *)P->y_wd32);
    D.ycheb = (const T *)(sizeof(T) == 8 ? (void *)P->y_cheb64 : (void *)P->y_cheb32);
    D.yww = P->y_ww;
    D.yself = P->y_self;
    D.ylam = P->y_lam;
    D.X = P->X; D.Y = P->Y; D.qs = P->qs; D.pside = P->d_pside;
    D.pstart = P->pstart; D.pcount = P->pcount; D.child0 = P->child0; D.parent = P->parent; D.col = P->colleague;
    D.proxy_slot = P->proxy_slot; D.local_slot = P->local_slot; D.psi_slot = P->psi_slot; D.blevel = P->blevel;
    D.anchor = P->anchor; D.bprob = P->bprob;
    D.bflags = P->bflags; D.bcenter = P->bcenter; D.anc_read = P->anc_read;
    const bool f64 = sizeof(T) == 8;
    D.c2p = (const T *)(f64 ? (void *)P->d_c2p : (void *)P->f_c2p);
    D.epw = (const T *)(f64 ? (void *)P->d_epw : (void *)P->f_epw);
    D.wd0 = (const T *)(f64 ? (void *)P->d_wd0 : (void *)P->f_wd0);
    D.gcheb = (const T *)(f64 ? (void *)P->d_gcheb : (void *)P->f_gcheb);
    D.gmono = (const T *)(f64 ? (void *)P->d_gmono : (void *)P->f_gmono);
    D.xcheb = (const T *)(f64 ? (void *)P->d_xcheb : (void *)P->f_xcheb);
    D.bary = (const T *)(f64 ? (void *)P->d_bary : (void *)P->f_bary);
    D.ew64 = P->d_ew; D.ww64 = P->d_ww; D.xcheb64 = P->d_xcheb; D.bary64 = P->d_bary;
    D.proxy = (T *)P->proxy; D.local = (T *)P->local; D.phi = (T *)P->phi; D.psi = (T *)P->psi;
    D.w0vals = (T *)P->w0vals;
    D.ufar = P->ufar; D.ures = P->ures;
    D.pwstride = (int64_t)t.nh * t.nn;
    return D;
}

size_t lds_root2(const Tables &t, int npmax)
{
    const size_t P = t.p;
    return sizeof(double) * (P * P + 2 * P * t.nwh + 2 * (size_t)t.nwn * t.nwh + 2 * P * t.nwh + 2 * P +
                             (size_t)std::max(npmax, 1) * 2 * P);
}

template <typename K>
void allow_lds2(K kernel, size_t bytes)
{
    int dev = 0, lim = 0;
    DMK_HIP(hipGetDevice(&dev));
    DMK_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if ((size_t)lim < bytes)
        throw Error{DMK_ERR_UNSUPPORTED, "device LDS per workgroup (" + std::to_string(lim) + " B) below the " +
                                             std::to_string(bytes) + " B a stage needs"};
    DMK_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

// Points a root leaf may hold (it is anterpolated inside the root kernel).
static int root_leaf_points(const Plan *Pl) { return (int)std::min<int64_t>(Pl->n, Pl->leaf_max); }

// persistent grid of the queue-fed upward kernel (set before any capture)
template <typename T, int P>
struct QGrid2 {
    static inline unsigned upward = 0;
    static void set()
    {
        if (!upward) upward = resident_blocks(k_upward2_q<T, P>, TPB, 0);
        (void)queue_wait_ticks();
    }
};

template <typename T, int P, int NF>
static void enqueue_core2(Plan *Pl, hipStream_t s, hipStream_t side)
{
    Dev2<T> D = make_dev2<T>(Pl);
    const auto &ll = Pl->ll;
    const int L = Pl->nlevels;
    if (side && Pl->nleaf) {
        DMK_HIP(hipEventRecord(Pl->ev_fork, s));
        DMK_HIP(hipStreamWaitEvent(side, Pl->ev_fork, 0));
        launch_residual2<T>(D, Pl, side);
        DMK_HIP(hipEventRecord(Pl->ev_join, side));
    }
    const bool levels = !Pl->queued;
    if (Pl->nfout && !levels) {  // one queue-fed launch over all levels
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        const WorkQ q = upward_queue(Pl);
        reset_queue(q.head, 4 + Pl->nfout, s);
        hipLaunchKernelGGL((k_upward2_q<T, P>), dim3((unsigned)std::min<int64_t>(Pl->nfout, QGrid2<T, P>::upward)),
                           dim3(TPB), 0, s, D, q);
    }
    for (int l = L - 1; l >= 0 && levels; --l) {
        int64_t m = ll.fout_off[l + 1] - ll.fout_off[l];
        if (!m) continue;
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        hipLaunchKernelGGL((k_upward2<T, P>), dim3((unsigned)m), dim3(TPB), 0, s, D, Pl->l_fout + ll.fout_off[l]);
    }
    {
        StageScope t(Pl, s, DMK_STAGE_ROOT);
        const int npmax = root_leaf_points(Pl);
        hipLaunchKernelGGL((k_root2<T, P>), dim3((unsigned)Pl->nprob), dim3(TPB), lds_root2(Pl->tab, npmax), s, D,
                           npmax);
    }
    if (Pl->nfout) {
        StageScope t(Pl, s, DMK_STAGE_PROXY2PW);
        hipLaunchKernelGGL((k_proxy2pw2<T, P, NF>), dim3((unsigned)Pl->nfout), dim3(TPB), 0, s, D, Pl->l_fout);
    }
    if (Pl->noct) {
        StageScope t(Pl, s, DMK_STAGE_PWSHIFT);
        const int64_t nm = (int64_t)Pl->tab.nh * Pl->tab.nn;
        const int nchunk = (int)((nm + TPB - 1) / TPB);
        const int64_t nb = (Pl->noct * nchunk + 7) / 8 * 8;
        hipLaunchKernelGGL((k_pwshift2<T>), dim3((unsigned)nb), dim3(TPB), 0, s, D, Pl->oct_dst, Pl->oct_src,
                           Pl->oct_level, Pl->oct_prob, Pl->noct, nchunk);
    }
    if (Pl->nanc && !levels) {  // one queue-fed launch over all levels
        StageScope t(Pl, s, DMK_STAGE_PW2GRID);
        const WorkQ q = local_queue(Pl);
        reset_queue(q.head, 4 + Pl->nanc, s);
        hipLaunchKernelGGL((k_local_pw2_q<T, P, NF>), dim3((unsigned)Pl->nanc), dim3(TPB), 0, s, D, q);
    }
    for (int l = 0; l < L && levels; ++l) {
        int64_t nan = ll.anc_off[l + 1] - ll.anc_off[l];
        if (!nan) continue;
        StageScope t(Pl, s, DMK_STAGE_PW2GRID);
        hipLaunchKernelGGL((k_local_pw2<T, P, NF>), dim3((unsigned)nan), dim3(TPB), 0, s, D,
                           Pl->l_anc + ll.anc_off[l], l);
    }
    if (Pl->nleaf) {
        {
            StageScope t(Pl, s, DMK_STAGE_LEAF);
            hipLaunchKernelGGL((k_leaf2<T, P>), dim3((unsigned)Pl->nanc), dim3(TPB), 0, s, D, Pl->l_anc,
                               Pl->anc_tbeg, Pl->anc_tgt);
        }
        if (side) {
            DMK_HIP(hipStreamWaitEvent(s, Pl->ev_join, 0));
        } else {
            StageScope t(Pl, s, DMK_STAGE_RESIDUAL);
            launch_residual2<T>(D, Pl, s);
        }
    }
}

template <typename T, int P, int NF>
static void run_eval2_t(Plan *Pl, const double *charges, double *pot, double *far_part, double *near_part,
                        hipStream_t s)
{
    const int64_t n = Pl->n;
    // the root kernel stages a root leaf's points: at most leaf_max of them
    allow_lds2(k_root2<T, P>, lds_root2(Pl->tab, root_leaf_points(Pl)));
    QGrid2<T, P>::set();
    {
        StageScope t(Pl, s, DMK_STAGE_GATHER);
        hipLaunchKernelGGL(k_gather_q2, dim3(nblk(n)), dim3(TPB), 0, s, charges, Pl->perm, n, Pl->qs);
    }
    const bool batched = (Pl->flags & DMK_FLAG_BATCHED) && !Pl->timing;
    if (batched) {
        if (!Pl->graph_exec) {
            hipGraph_t g = nullptr;
            DMK_HIP(hipStreamBeginCapture(Pl->cap_stream, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_core2<T, P, NF>(Pl, Pl->cap_stream, Pl->side_stream);
            } catch (...) {
                (void)hipStreamEndCapture(Pl->cap_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            DMK_HIP(hipStreamEndCapture(Pl->cap_stream, &g));
            DMK_HIP(hipGraphInstantiate(&Pl->graph_exec, g, nullptr, nullptr, 0));
            DMK_HIP(hipGraphDestroy(g));
        }
        DMK_HIP(hipGraphLaunch(Pl->graph_exec, s));
    } else {
        enqueue_core2<T, P, NF>(Pl, s, nullptr);
    }
    {
        StageScope t(Pl, s, DMK_STAGE_FINALIZE);
        hipLaunchKernelGGL(k_finalize2, dim3(nblk(n)), dim3(TPB), 0, s, Pl->ufar, Pl->ures, Pl->perm, n, pot,
                           far_part, near_part);
    }
    DMK_HIP(hipGetLastError());
}

void run_eval2(Plan *P, const double *charges, double *pot, double *far_part, double *near_part, hipStream_t s)
{
    if (P->n == 0) return;
    const bool f64 = P->precision == DMK_FP64;
    switch (P->p) {
    case 18:
        if (f64) run_eval2_t<double, 18, 12>(P, charges, pot, far_part, near_part, s);
        else run_eval2_t<float, 18, 12>(P, charges, pot, far_part, near_part, s);
        break;
    case 15:
        if (f64) run_eval2_t<double, 15, 10>(P, charges, pot, far_part, near_part, s);
        else run_eval2_t<float, 15, 10>(P, charges, pot, far_part, near_part, s);
        break;
    case 9:
        if (f64) run_eval2_t<double, 9, 6>(P, charges, pot, far_part, near_part, s);
        else run_eval2_t<float, 9, 6>(P, charges, pot, far_part, near_part, s);
        break;
    default:
        throw Error{DMK_ERR_UNSUPPORTED, "no kernels for this proxy order"};
    }
}

void workspace_layout2(Plan *P, std::vector<WsItem> &items)
{
    const Tables &t = P->tab;
    const size_t el = (P->precision == DMK_FP64) ? sizeof(double) : sizeof(float);
    const int64_t p2 = (int64_t)t.p * t.p;
    const int64_t nm = (int64_t)t.nh * t.nn;
    auto add = [&](void *field, int64_t cnt, size_t sz) {
        items.push_back({(void **)field, (size_t)std::max<int64_t>(cnt, 1) * sz});
    };
    add(&P->qs, P->n, 8);
    add(&P->ufar, P->n, 8);
    add(&P->ures, P->n, 8);
    add(&P->proxy, P->nfout * p2, el);
    add(&P->local, P->nanc * p2, el);
    add(&P->phi, 2 * P->nfout * nm, el);
    add(&P->psi, 2 * P->nfin * nm, el);
    add(&P->w0vals, P->nprob * p2, el);
    add(&P->qctl, queue_ctl_words(P), 4);
}

}  // namespace dmk
