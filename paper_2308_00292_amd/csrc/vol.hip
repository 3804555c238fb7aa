// Volume potential on gfx950: u(x) = int_{B_0} rho(y) / (4 pi |x - y|) dy on
// the unit cube, at the Chebyshev nodes of a density-adaptive tree (Sec. 3.6,
// "Modification of DMK for continuous sources").
//
// Split: the Gaussian multilevel form of Sec. 3.2 (eqs. mlks, kerneldef,
// deltavalue), sigma_l = 2^-l / sqrt(log(1/eps)); its plane-wave weights obey
// w_l = 2^l w_0 like the PSWF ones, so the far-field stages of the point code
// (root window, outgoing and incoming plane waves, local values of the
// anchors) run unchanged on Gaussian tables.  What the volume code adds:
//
//   host       the tree that resolves rho (calls of the density callback,
//              Chebyshev tail test, 2:1 balance), handed to the point-code
//              tree builder as its node set with leaf capacity q^3 and the
//              unit cube as root, so that builder's leaves are these leaves.
//   k_vol_upward  proxy charges of every non-leaf box: leaf children from
//              their density (Gauss-Legendre weights times rho at the Legendre
//              nodes, anterpolated to the parent grid: one p x q matrix per
//              axis and child side), non-leaf children by the child->parent
//              matrices.
//   k_vol_leaf the anchor's local polynomial at the leaf's q^3 nodes (three
//              q x p mode products).
//   k_vol_near residual R_L of every source leaf in the target leaf's gather
//              list as a sum of Gaussians (Gauss-Legendre in log t), each a
//              product of three q x q matrices; the Gaussians narrower than
//              1/t_a over R^3 through rho + Lap rho/(4t^2) + Lap^2 rho/(32t^4)
//              of the target's polynomial (Sec. 4.4).
//   k_vol_finalize  u = (far + near) / (4 pi).
//
// HBM layout: rho and u leaf-major in Morton order, q^3 per leaf with the
// z index fastest; per-box p^3 grids and plane waves as in the point code.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_set>

#include "dmk_internal.h"
#include "queue.h"
#include "tiles.h"

namespace dmk {

namespace {

constexpr int VQ = 8;  // leaf grid order built

// ---------------------------------------------------------------- host tree
struct Cell {
    int32_t l, c[3];
};

uint64_t spread_bits(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

// Morton key at 21 bits per axis (x most significant within a bit triple)
uint64_t cell_key(const Cell &a)
{
    const int sh = 21 - a.l;
    return (spread_bits((uint64_t)a.c[0] << sh) << 2) | (spread_bits((uint64_t)a.c[1] << sh) << 1) |
           spread_bits((uint64_t)a.c[2] << sh);
}

// unique per (level, cell): the level above the level's own key bits
uint64_t cell_id(int l, int64_t x, int64_t y, int64_t z)
{
    Cell a{l, {(int32_t)x, (int32_t)y, (int32_t)z}};
    return ((uint64_t)l << 58) | (cell_key(a) >> (3 * (21 - l)));
}

// Chebyshev coefficients c_k = (2 - [k = 0]) / q sum_a f(x_a) T_k(x_a), x_a =
// cos(pi (a + 1/2) / q), along one axis of a q^3 block (stride st)
void dct_axis(int q, double *f, int st0, int st1, int st2)
{
    std::vector<double> C((size_t)q * q), tmp(q);
    for (int k = 0; k < q; ++k)
        for (int a = 0; a < q; ++a) C[k * q + a] = (k ? 2.0 : 1.0) / q * std::cos(k * M_PI * (a + 0.5) / q);
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            double *b = f + i * st1 + j * st2;
            for (int k = 0; k < q; ++k) {
                double s = 0.0;
                for (int a = 0; a < q; ++a) s += C[k * q + a] * b[a * st0];
                tmp[k] = s;
            }
            for (int k = 0; k < q; ++k) b[k * st0] = tmp[k];
        }
}

// refinement test: sum of |c_ijk| with max(i,j,k) >= q-2
double cheb_tail(int q, std::vector<double> f)
{
    dct_axis(q, f.data(), q * q, q, 1);
    dct_axis(q, f.data(), q, q * q, 1);
    dct_axis(q, f.data(), 1, q * q, q);
    double s = 0.0;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k)
                if (i >= q - 2 || j >= q - 2 || k >= q - 2) s += std::fabs(f[(i * q + j) * q + k]);
    return s;
}

void cell_nodes(int q, const Cell &b, double *xyz)
{
    const double s = std::ldexp(1.0, -b.l);
    double cen[3];
    for (int d = 0; d < 3; ++d) cen[d] = -0.5 + (b.c[d] + 0.5) * s;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                const int ix[3] = {i, j, k};
                double *o = xyz + 3 * ((i * q + j) * q + k);
                for (int d = 0; d < 3; ++d) o[d] = cen[d] + 0.5 * s * std::cos(M_PI * (ix[d] + 0.5) / q);
            }
}

// a feature point inside the box asks for a side below the box's
bool feature_split(const Cell &b, int32_t nfeat, const double *feat)
{
    const double s = std::ldexp(1.0, -b.l);
    for (int32_t f = 0; f < nfeat; ++f) {
        const double *F = feat + 4 * (size_t)f;
        if (!(F[3] < s)) continue;
        bool in = true;
        for (int d = 0; d < 3; ++d) {
            const double lo = -0.5 + b.c[d] * s;
            in = in && F[d] >= lo && F[d] < lo + s;
        }
        if (in) return true;
    }
    return false;
}

std::vector<Cell> build_vol_tree(int q, double tol, double rho_scale, int min_level, int max_level, int32_t nfeat,
                                 const double *feat, dmk_density_fn fn, void *ctx)
{
    const int q3 = q * q * q;
    std::vector<Cell> leaves, cur{Cell{0, {0, 0, 0}}};
    for (int l = 0; !cur.empty(); ++l) {
        std::vector<char> split(cur.size(), 0);
        if (l < max_level) {
            if (l < min_level) {
                std::fill(split.begin(), split.end(), 1);
            } else {
                std::vector<double> xyz(cur.size() * q3 * 3), f(cur.size() * q3);
                for (size_t b = 0; b < cur.size(); ++b) cell_nodes(q, cur[b], xyz.data() + b * q3 * 3);
                fn((int64_t)(cur.size() * q3), xyz.data(), f.data(), ctx);
                for (size_t b = 0; b < cur.size(); ++b) {
                    std::vector<double> fb(f.begin() + b * q3, f.begin() + (b + 1) * q3);
                    for (double v : fb)
                        if (!std::isfinite(v)) throw Error{DMK_ERR_ARG, "density returned a non-finite value"};
                    split[b] = feature_split(cur[b], nfeat, feat) || cheb_tail(q, fb) > tol * rho_scale;
                }
            }
        }
        std::vector<Cell> nxt;
        for (size_t b = 0; b < cur.size(); ++b) {
            if (!split[b]) {
                leaves.push_back(cur[b]);
                continue;
            }
            for (int o = 0; o < 8; ++o)
                nxt.push_back(Cell{l + 1, {2 * cur[b].c[0] + ((o >> 2) & 1), 2 * cur[b].c[1] + ((o >> 1) & 1),
                                           2 * cur[b].c[2] + (o & 1)}});
        }
        cur.swap(nxt);
    }
    // minimal 2:1 balance: a leaf touching a leaf two or more levels finer is split
    for (;;) {
        std::unordered_set<uint64_t> have;
        have.reserve(leaves.size() * 2);
        for (const Cell &a : leaves) have.insert(cell_id(a.l, a.c[0], a.c[1], a.c[2]));
        std::unordered_set<uint64_t> mark;
        for (const Cell &a : leaves) {
            if (a.l < 2) continue;
            const int64_t lim = int64_t(1) << a.l;
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        if (!dx && !dy && !dz) continue;
                        const int64_t n[3] = {a.c[0] + dx, a.c[1] + dy, a.c[2] + dz};
                        if (n[0] < 0 || n[1] < 0 || n[2] < 0 || n[0] >= lim || n[1] >= lim || n[2] >= lim) continue;
                        for (int up = 0; up <= a.l; ++up) {
                            const uint64_t id = cell_id(a.l - up, n[0] >> up, n[1] >> up, n[2] >> up);
                            if (have.count(id)) {
                                if (up >= 2) mark.insert(id);
                                break;
                            }
                        }
                    }
        }
        if (mark.empty()) break;
        std::vector<Cell> nl;
        nl.reserve(leaves.size() + 7 * mark.size());
        for (const Cell &a : leaves) {
            if (!mark.count(cell_id(a.l, a.c[0], a.c[1], a.c[2]))) {
                nl.push_back(a);
                continue;
            }
            for (int o = 0; o < 8; ++o)
                nl.push_back(Cell{a.l + 1, {2 * a.c[0] + ((o >> 2) & 1), 2 * a.c[1] + ((o >> 1) & 1),
                                            2 * a.c[2] + (o & 1)}});
        }
        leaves.swap(nl);
    }
    std::sort(leaves.begin(), leaves.end(), [](const Cell &a, const Cell &b) { return cell_key(a) < cell_key(b); });
    return leaves;
}

// ------------------------------------------------------------- host tables
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), d = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            d = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / d;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        d = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * d * d);
    }
}

// Lagrange basis of the n first-kind Chebyshev nodes at x (barycentric)
void cheb_lagrange(int n, double x, double *out)
{
    double den = 0.0;
    for (int a = 0; a < n; ++a) {
        const double xa = std::cos(M_PI * (a + 0.5) / n);
        const double wa = ((a & 1) ? -1.0 : 1.0) * std::sin((2 * a + 1) * M_PI / (2.0 * n));
        if (x == xa) {
            for (int b = 0; b < n; ++b) out[b] = (b == a) ? 1.0 : 0.0;
            return;
        }
        out[a] = wa / (x - xa);
        den += out[a];
    }
    for (int a = 0; a < n; ++a) out[a] /= den;
}

// Gaussian split tables over a copy of the PSWF ones (same p, n_f, grids):
// D_0 weights (h_0/2pi)^3 Dhat_0(h_0|m|), root window weights with the
// Gaussian factor, spacing h_W = 2 pi / (2 sqrt 3 + 2), n_W = 14.
void gauss_tables(Tables *t, double tol)
{
    const double s0 = 1.0 / std::sqrt(std::log(1.0 / tol)), s1 = 0.5 * s0;
    const int nf = t->nf, p = t->p;
    {
        const double h = 2.0 * M_PI / 3.0, fac = std::pow(h / (2.0 * M_PI), 3);
        const int maxk2 = 3 * nf * nf;
        std::vector<double> memo(maxk2 + 1);
        memo[0] = fac * M_PI * (s0 * s0 - s1 * s1);
        for (int k2 = 1; k2 <= maxk2; ++k2) {
            const double k = h * std::sqrt((double)k2);
            // 4 pi (e^{-k^2 s1^2/4} - e^{-k^2 s0^2/4}) / k^2
            memo[k2] = fac * 4.0 * M_PI * std::exp(-0.25 * k * k * s1 * s1) *
                       (-std::expm1(-0.25 * k * k * (s0 * s0 - s1 * s1))) / (k * k);
        }
        for (int m1 = -nf; m1 <= nf; ++m1)
            for (int m3 = 0; m3 <= nf; ++m3)
                for (int m2 = -nf; m2 <= nf; ++m2)
                    t->wd0[((size_t)(m1 + nf) * t->nh + m3) * t->nn + (m2 + nf)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
    }
    const int nw = 14;
    const double hw = 2.0 * M_PI / (2.0 * std::sqrt(3.0) + 2.0);
    t->nw = nw;
    t->nwn = 2 * nw + 1;
    t->nwh = nw + 1;
    t->prm.nw = nw;
    t->prm.hw = hw;
    t->ew.assign((size_t)t->nwn * p * 2, 0.0);
    for (int m = -nw; m <= nw; ++m)
        for (int j = 0; j < p; ++j) {
            const double ph = -hw * m * 0.5 * t->xcheb[j];
            t->ew[((size_t)(m + nw) * p + j) * 2 + 0] = std::cos(ph);
            t->ew[((size_t)(m + nw) * p + j) * 2 + 1] = std::sin(ph);
        }
    const double A = 1.0 + std::sqrt(3.0), fac = std::pow(hw / (2.0 * M_PI), 3);
    const int maxk2 = 3 * nw * nw;
    std::vector<double> memo(maxk2 + 1);
    memo[0] = fac * 2.0 * M_PI * A * A;
    for (int k2 = 1; k2 <= maxk2; ++k2) {
        const double k = hw * std::sqrt((double)k2), sn = std::sin(0.5 * k * A);
        memo[k2] = fac * 8.0 * M_PI * sn * sn / (k * k) * std::exp(-0.25 * k * k * s0 * s0);
    }
    t->ww.assign((size_t)t->nwh * t->nwn * t->nwn, 0.0);
    for (int m3 = 0; m3 <= nw; ++m3)
        for (int m2 = -nw; m2 <= nw; ++m2)
            for (int m1 = -nw; m1 <= nw; ++m1)
                t->ww[((size_t)m3 * t->nwn + (m2 + nw)) * t->nwn + (m1 + nw)] = memo[m1 * m1 + m2 * m2 + m3 * m3];
}

// ------------------------------------------------------------ device view
template <typename T>
struct VDev {
    const int32_t *child0, *blevel, *proxy_slot, *local_slot, *anchor, *box2v, *vlevel, *vijk;
    const uint8_t *bflags;
    const double *bcenter;
    const T *c2p, *xcheb, *bary, *v1;
    const double *xq, *bq, *d2, *tgl, *tglw, *egl, *eglw;
    int ngl;
    double tpan_w, tau_a, sqL;
    const double *rho;
    T *proxy;
    const T *local;
    double *ufar, *unear;
};

template <typename T>
VDev<T> make_vdev(Plan *P)
{
    VDev<T> D;
    const bool f64 = sizeof(T) == 8;
    D.child0 = P->child0;
    D.blevel = P->blevel;
    D.proxy_slot = P->proxy_slot;
    D.local_slot = P->local_slot;
    D.anchor = P->anchor;
    D.box2v = P->vol.box2v;
    D.vlevel = P->vol.d_level;
    D.vijk = P->vol.d_ijk;
    D.bflags = P->bflags;
    D.bcenter = P->bcenter;
    D.c2p = (const T *)(f64 ? (void *)P->d_c2p : (void *)P->f_c2p);
    D.xcheb = (const T *)(f64 ? (void *)P->d_xcheb : (void *)P->f_xcheb);
    D.bary = (const T *)(f64 ? (void *)P->d_bary : (void *)P->f_bary);
    D.v1 = (const T *)(f64 ? (void *)P->vol.d_v1 : (void *)P->vol.f_v1);
    D.xq = P->vol.d_xq;
    D.bq = P->vol.d_bq;
    D.d2 = P->vol.d_d2;
    D.tgl = P->vol.d_tgl;
    D.tglw = P->vol.d_tglw;
    D.egl = P->vol.d_egl;
    D.eglw = P->vol.d_eglw;
    D.ngl = P->vol.tpan_gl;
    D.tpan_w = P->vol.tpan_w;
    D.tau_a = P->vol.tau_a;
    D.sqL = P->vol.sqL;
    D.rho = nullptr;
    D.proxy = (T *)P->proxy;
    D.local = (const T *)P->local;
    D.ufar = P->vol.ufar;
    D.unear = P->vol.unear;
    return D;
}

// ------------------------------------------------------------------ kernels
// node coordinates of every leaf, [n][3]
__global__ void __launch_bounds__(TPB) k_vol_nodes(const int32_t *lev, const int32_t *ijk, const double *xq, int q,
                                                   int64_t n, double *xyz)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    const int q3 = q * q * q;
    const int64_t b = i / q3;
    const int r = (int)(i % q3);
    const int ix[3] = {r / (q * q), (r / q) % q, r % q};
    const double s = ldexp(1.0, -lev[b]);
    for (int d = 0; d < 3; ++d) xyz[3 * i + d] = -0.5 + (ijk[3 * b + d] + 0.5) * s + 0.5 * s * xq[ix[d]];
}

// leaf box -> volume leaf, from the point-code tree over the nodes: every
// leaf box must hold exactly the q^3 nodes of one volume leaf
__global__ void __launch_bounds__(TPB) k_vol_map(const int32_t *leaves, int64_t nleaf, const int32_t *pstart,
                                                 const int32_t *pcount, const int32_t *perm, int q3, int32_t *box2v,
                                                 unsigned long long *bad)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nleaf) return;
    const int32_t B = leaves[i];
    const int32_t c = pcount[B], s0 = pstart[B];
    bool ok = (c == q3);
    const int32_t v = ok ? perm[s0] / q3 : -1;
    for (int k = 0; ok && k < q3; ++k) ok = (perm[s0 + k] / q3 == v);
    box2v[B] = ok ? v : -1;
    if (!ok) atomicAdd(bad, 1ull);
}

template <int P, int Q>
struct VolLds {
    static constexpr int P2 = P * P, P3 = P2 * P, Q3 = Q * Q * Q;
    static constexpr int up_work = (2 * P3 > Q3 + Q * Q * P + Q * P2) ? 2 * P3 : Q3 + Q * Q * P + Q * P2;
    static size_t up(size_t el) { return el * (2 * P2 + 2 * P * Q + up_work); }
    static size_t leaf(size_t el) { return el * (P3 + P2 * Q + P * Q * Q + 3 * Q * P + 2 * P); }
    static constexpr int JB = 5;  // Gaussians per pass of the near-field kernel (one panel at tol 1e-3)
    static constexpr int JB6 = 10;  // the same at tol 1e-6 (30 or 40 Gaussians per pair)
    // source densities staged per batch: seven with five waves (FP32: six
    // blocks per CU), nine with ten (a z group of nine colleagues in one batch)
    static constexpr int nb(int jb) { return jb == 5 ? 7 : 9; }
    // NB source blocks, then a [q^2][q+1] regrouping buffer per wave; the
    // epilogue reuses them for the partial sums and the Laplacians
    static size_t near(size_t el, int jb = JB)
    {
        const size_t main = el * (nb(jb) * Q3 + jb * Q * Q * (Q + 1)), epi = sizeof(double) * (jb * Q3 + 3 * Q3 + Q * Q);
        return main > epi ? main : epi;
    }
};

// proxy charges of the non-leaf boxes of one level
// COH: the box's F_out children were computed by the same launch (queue-fed)
template <typename T, int P, int Q, bool COH>
__device__ __forceinline__ void vol_upward_box(const VDev<T> &D, const int32_t Pb)
{
    constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
    constexpr int RM = Tiles<P>::RM, RN = Tiles<P>::RN, ZM = Tiles<P>::ZM, ZN = Tiles<P>::ZN;
    extern __shared__ __align__(16) unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    T *Am = sm;              // [2][p][p] child -> parent
    T *Vm = Am + 2 * P2;     // [2][p][q] leaf density -> parent
    T *w0 = Vm + 2 * P * Q;  // work
    for (int t = threadIdx.x; t < 2 * P2; t += TPB) Am[t] = D.c2p[t];
    for (int t = threadIdx.x; t < 2 * P * Q; t += TPB) Vm[t] = D.v1[t];
    T acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = T(0);
    const double sc = ldexp(1.0, -3 * (D.blevel[Pb] + 2));  // (s_child / 2)^3
    __syncthreads();
    for (int k = 0; k < 8; ++k) {
        const int32_t C = D.child0[Pb] + k;
        const int bx = (k >> 2) & 1, by = (k >> 1) & 1, bz = k & 1;
        if (D.bflags[C] & 2) {
            const T *src = D.proxy + (int64_t)D.proxy_slot[C] * P3;
            T *t1 = w0, *t2 = w0 + P3;
            __syncthreads();
            copy_to_lds<COH, TPB>(t2, src, P3);
            __syncthreads();
            gemm<T, ZM, ZN, false>(1, P2, P, P, t2, 0, P, 1, Am + bz * P2, 0, 1, P, t1, 0, P, 1);
            __syncthreads();
            gemm<T, ZM, ZN, false>(P, P, P, P, Am + by * P2, 0, P, 1, t1, P2, P, 1, t2, P2, P, 1);
            __syncthreads();
            gemm_regs<T, RM, RN>(P, P2, P, Am + bx * P2, P, 1, t2, P2, 1, acc);
        } else {
            // leaf child: rho on its q^3 nodes -> parent grid
            const double *rho = D.rho + (int64_t)D.box2v[C] * Q3;
            T *r = w0, *t1 = r + Q3, *t2 = t1 + Q2 * P;
            __syncthreads();
            for (int t = threadIdx.x; t < Q3; t += TPB) r[t] = (T)(rho[t] * sc);
            __syncthreads();
            // z: t1[(i0 i1)][a2] = sum_i2 r[(i0 i1)][i2] V_z[a2][i2]
            gemm<T, ZM, ZN, false>(1, Q2, P, Q, r, 0, Q, 1, Vm + bz * P * Q, 0, 1, Q, t1, 0, P, 1);
            __syncthreads();
            // y: t2[i0][a1][a2] = sum_i1 V_y[a1][i1] t1[i0][i1][a2]
            gemm<T, ZM, ZN, false>(Q, P, P, Q, Vm + by * P * Q, 0, Q, 1, t1, Q * P, P, 1, t2, P2, P, 1);
            __syncthreads();
            // x: acc[a0][(a1 a2)] += sum_i0 V_x[a0][i0] t2[i0][(a1 a2)]
            gemm_regs<T, RM, RN>(P, P2, Q, Vm + bx * P * Q, Q, 1, t2, P2, 1, acc);
        }
    }
    store_tiles<T, P, COH>(acc, D.proxy + (int64_t)D.proxy_slot[Pb] * P3);
}

// one level's non-leaf boxes, one workgroup per box
template <typename T, int P, int Q>
__global__ void __launch_bounds__(TPB) k_vol_upward(VDev<T> D, const int32_t *list)
{
    vol_upward_box<T, P, Q, false>(D, list[blockIdx.x]);
}

// the non-leaf boxes of every level, finest first, from the work queue (a
// box waits for its non-leaf children)
template <typename T, int P, int Q>
__global__ void __launch_bounds__(TPB) k_vol_upward_q(VDev<T> D, WorkQ q)
{
    queue_loop(
        q,
        [&](int32_t Pb) {
            if (threadIdx.x < 8) {
                const int32_t C = D.child0[Pb] + threadIdx.x;
                if (D.bflags[C] & 2) wait_done(q, C);
            }
        },
        [&](int32_t Pb) { vol_upward_box<T, P, Q, true>(D, Pb); });
}

// far field at the nodes of each leaf from its anchor's local values
template <typename T, int P, int Q>
__global__ void __launch_bounds__(TPB) k_vol_leaf(VDev<T> D, const int32_t *leaves)
{
    constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q;
    extern __shared__ __align__(16) unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    T *v = sm;               // p^3 local values of the anchor
    T *t1 = v + P3;          // [p][p][q]
    T *t2 = t1 + P2 * Q;     // [p][q][q]
    T *U = t2 + P * Q2;      // [3][q][p] Lagrange rows of the anchor grid at the nodes
    T *xc = U + 3 * Q * P, *bw = xc + P;
    const int32_t B = leaves[blockIdx.x];
    const int32_t A = D.anchor[B];
    const int32_t vB = D.box2v[B];
    const T *src = D.local + (int64_t)D.local_slot[A] * P3;
    for (int t = threadIdx.x; t < P3; t += TPB) v[t] = src[t];
    for (int t = threadIdx.x; t < P; t += TPB) {
        xc[t] = D.xcheb[t];
        bw[t] = D.bary[t];
    }
    __syncthreads();
    const double sB = ldexp(1.0, -D.blevel[B]), sA = ldexp(1.0, -D.blevel[A]);
    for (int r = threadIdx.x; r < 3 * Q; r += TPB) {
        const int d = r / Q, i = r % Q;
        const double x = D.bcenter[3 * (int64_t)B + d] + 0.5 * sB * D.xq[i];
        const T xi = (T)(2.0 * (x - D.bcenter[3 * (int64_t)A + d]) / sA);
        T row[P];
        lagrange_row<T>(P, xc, bw, xi, row);
#pragma unroll
        for (int a = 0; a < P; ++a) U[(d * Q + i) * P + a] = row[a];
    }
    __syncthreads();
    // z: t1[(a0 a1)][i2] = sum_a2 v[(a0 a1)][a2] U_z[i2][a2]
    gemm<T, 3, 2, false>(1, P2, Q, P, v, 0, P, 1, U + 2 * Q * P, 0, 1, P, t1, 0, Q, 1);
    __syncthreads();
    // y: t2[a0][i1][i2] = sum_a1 U_y[i1][a1] t1[a0][a1][i2]
    gemm<T, 2, 2, false>(P, Q, Q, P, U + Q * P, 0, P, 1, t1, P * Q, Q, 1, t2, Q2, Q, 1);
    __syncthreads();
    // x: u[i0][(i1 i2)] = sum_a0 U_x[i0][a0] t2[a0][(i1 i2)]
    const int o = threadIdx.x;
    for (int k = o; k < Q * Q2; k += TPB) {
        const int i0 = k / Q2, r = k % Q2;
        double s = 0.0;
        for (int a = 0; a < P; ++a) s += (double)U[i0 * P + a] * (double)t2[a * Q2 + r];
        D.ufar[(int64_t)vB * Q * Q2 + k] = s;
    }
}

// 1-D factors of the near field for a unit source box, one row (class c,
// Gaussian j, target node a) per thread:
//   G[a][b] = (1/2) int_{-1}^{1} exp(-(xi_a - eta)^2 tau_j^2) L_b(eta) d eta,
//   xi_a = 2 delta + 2^-k x_a, tau_j = t_j / 2,
// t_j the Gauss-Legendre nodes in log t of the class's panels; 32-point
// Gauss-Legendre on the part of [-1,1] within 7/tau of xi (the rest is below
// e^-49), with L_b = (1/q) [1 + 2 sum_k T_k(x_b) T_k(eta)] accumulated as
// Chebyshev moments.  Row a = 0 also writes the weight
// (2/sqrt pi) t_j (h/2) w_j of the Gaussian.
__global__ void __launch_bounds__(TPB) k_vol_gtab(const double *xq, const double *tgl, const double *tglw,
                                                  const double *egl, const double *eglw, int ngl, double tpan_w,
                                                  double tau_a, double sqL, int q, int64_t nk, const int32_t *kk,
                                                  const double *kd, const int32_t *kng, const int64_t *kbase,
                                                  int nfit, const double *fit, int64_t rows, double *gtab,
                                                  double *gw)
{
    const int64_t r = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (r >= rows) return;
    const int64_t g = r / q;
    const int a = (int)(r % q);
    int64_t lo = 0, hi = nk - 1;
    while (lo < hi) {
        const int64_t m = (lo + hi + 1) / 2;
        if (kbase[m] <= g) lo = m;
        else hi = m - 1;
    }
    const int64_t c = lo;
    const int j = (int)(g - kbase[c]), k = kk[c];
    const double u0 = log(sqL), u1 = log(tau_a) + k * log(2.0);
    const int npan = (kng[c] - nfit) / ngl;
    const double hp = (u1 - u0) / npan;
    const int pan = j / ngl, gi = j % ngl;
    const bool fitted = j >= npan * ngl;  // PSWF split: the fitted Gaussians follow the panels
    const double tj = fitted ? fit[j - npan * ngl] : exp(u0 + hp * (pan + 0.5 * (tgl[gi] + 1.0)));
    const double tau = 0.5 * tj;
    const double xi = 2.0 * kd[c] + ldexp(1.0, -k) * xq[a];
    const double lo_ = fmax(-1.0, xi - 7.0 / tau), hi_ = fmin(1.0, xi + 7.0 / tau);
    double cf[16];
    for (int m = 0; m < q; ++m) cf[m] = 0.0;
    if (hi_ > lo_) {
        const double hc = 0.5 * (lo_ + hi_), hr = 0.5 * (hi_ - lo_);
        for (int n = 0; n < 32; ++n) {
            const double eta = hc + hr * egl[n];
            const double dd = (xi - eta) * tau;
            const double wgt = exp(-dd * dd) * hr * eglw[n];
            double t0 = 1.0, t1 = eta;
            cf[0] += wgt;
            if (q > 1) cf[1] += wgt * eta;
            for (int m = 2; m < q; ++m) {
                const double t2 = 2.0 * eta * t1 - t0;
                cf[m] += wgt * t2;
                t0 = t1;
                t1 = t2;
            }
        }
    }
    double *out = gtab + (g * q + a) * q;
    for (int b = 0; b < q; ++b) {
        double s = cf[0];
        for (int m = 1; m < q; ++m) s += 2.0 * cos(m * M_PI * (b + 0.5) / q) * cf[m];
        out[b] = 0.5 * s / q;
    }
    if (a == 0) gw[g] = fitted ? fit[nfit + j - npan * ngl] : 2.0 / sqrt(M_PI) * tj * 0.5 * hp * tglw[gi];
}

__global__ void __launch_bounds__(TPB) k_vol_tof32(const double *src, float *dst, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// Near field of each target leaf: for every source leaf T of its gather list
// that survives the pruning, sum over the class's Gaussians of
// s_T^2 w_j (G_x (x) G_y (x) G_z) rho_T, then the asymptotic part from the
// target's own polynomial.  FP64.
//
// One wavefront per Gaussian of a log-t panel (5 waves, the panel's 5 nodes;
// every class has whole panels).  The 8 x 8 factors are wave-uniform and
// read-only, so they come through the scalar cache and feed the FMAs as
// scalar operands.  The entries of a gather list arrive sorted by (z class,
// y class, x class): x passes are summed over the sources of a (y, z) group,
// y passes over the groups of a z class, and one z pass closes each z
// class (27 + 9 + 3 passes per Gaussian for the 27 colleagues of a uniform
// region instead of 81).  Lane L holds one row of the 8^3 block in each pass
// (rows (i1 i2), then (a i2), then (a b)); a wave-private LDS buffer
// regroups between passes.  The sources' densities are staged in LDS in
// batches of NB.
// T: precision of the factor products and their sums (FP64, or FP32 for
// mixed-precision plans); the asymptotic part and the output stay FP64.
// FP32 with five waves per block: registers capped for eight waves per SIMD
// (62 VGPRs instead of 82, no spills), so six blocks fit a CU as its LDS allows
template <typename T, int Q, int JB>
__global__ void __launch_bounds__(Q * Q * JB, (sizeof(T) == 4 && JB == 5) ? 8 : 1)
    k_vol_near(VDev<double> D, const int32_t *__restrict__ leaves, const int32_t *__restrict__ nl_off,
               const int32_t *__restrict__ nl_src, const int32_t *__restrict__ esrc, const int32_t *__restrict__ pk,
               const T *__restrict__ gtab, const double *__restrict__ gw)
{
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q, NB = VolLds<18, Q>::nb(JB), RS = Q + 1, NT = JB * Q2;
    static_assert(Q2 == 64, "one wavefront per Gaussian, one lane per row");
    extern __shared__ __align__(16) double vsm[];
    T *slot = reinterpret_cast<T *>(vsm);  // [NB][q^3] source densities
    T *wb = slot + NB * Q3;                // per wave: [q^2][RS] regrouping buffer
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / Q2);  // wave = Gaussian of the panel
    const int L = tid % Q2;
    T *buf = wb + w * Q2 * RS;
    const int64_t li = blockIdx.x;
    const int32_t B = leaves[li];
    const int32_t vB = D.box2v[B];
    const double sB = ldexp(1.0, -D.blevel[B]);
    T acc[Q];  // lane (a b): acc[c]
#pragma unroll
    for (int c = 0; c < Q; ++c) acc[c] = T(0);
    const int eend = nl_off[li + 1];
    for (int e = nl_off[li]; e < eend;) {
        if (pk[4 * (int64_t)e] < 0) break;  // pruned entries come last
        int ez = e;
        for (;;) {  // end of this z class
            const int fl = pk[4 * (int64_t)ez + 3];
            ++ez;
            if (fl & 2) break;
        }
        const int32_t kx0 = pk[4 * (int64_t)e], kzc = pk[4 * (int64_t)e + 2];
        const double sT = ldexp(1.0, -D.blevel[nl_src[e]]);
        const int ng = pk[4 * (int64_t)e + 3] >> 2;
        for (int j0 = 0; j0 < ng; j0 += JB) {
            const int64_t j = j0 + w;
            const T wj = (T)(gw[kx0 + j] * sT * sT);
            T xa[Q], ya[Q];  // lane (i1 i2): xa[a]; lane (a i2): ya[b]
#pragma unroll
            for (int k = 0; k < Q; ++k) xa[k] = ya[k] = T(0);
            for (int b0 = e; b0 < ez; b0 += NB) {
                const int nb = min(NB, ez - b0);
                __syncthreads();
                for (int t = tid; t < nb * Q3; t += NT) {
                    const int sidx = t / Q3;
                    slot[t] = (T)D.rho[(int64_t)esrc[b0 + sidx] * Q3 + t % Q3];
                }
                __syncthreads();
                for (int sidx = 0; sidx < nb; ++sidx) {
                    const int64_t es = b0 + sidx;
                    // x: xa[a] += sum_i0 G_x[a][i0] rho[i0][(i1 i2)]
                    const T *gx = gtab + (pk[4 * es] + j) * Q2;
                    const T *rs = slot + sidx * Q3;
                    T r[Q];
#pragma unroll
                    for (int i0 = 0; i0 < Q; ++i0) r[i0] = rs[i0 * Q2 + L];
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        T s = T(0);
#pragma unroll
                        for (int i0 = 0; i0 < Q; ++i0) s += gx[a * Q + i0] * r[i0];
                        xa[a] += s;
                    }
                    if (pk[4 * es + 3] & 1) {
                        // end of a (y, z) group: ya[b] += sum_i1 G_y[b][i1] X[a][i1][i2]
                        const T *gy = gtab + (pk[4 * es + 1] + j) * Q2;
#pragma unroll
                        for (int a = 0; a < Q; ++a) buf[L * RS + a] = xa[a];
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        const int a = L / Q, i2 = L % Q;
                        T y[Q];
#pragma unroll
                        for (int i1 = 0; i1 < Q; ++i1) y[i1] = buf[(i1 * Q + i2) * RS + a];
#pragma unroll
                        for (int bb = 0; bb < Q; ++bb) {
                            T s = T(0);
#pragma unroll
                            for (int i1 = 0; i1 < Q; ++i1) s += gy[bb * Q + i1] * y[i1];
                            ya[bb] += s;
                        }
#pragma unroll
                        for (int k = 0; k < Q; ++k) xa[k] = T(0);
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
            // end of the z class: acc[c] += w_j sum_i2 G_z[c][i2] Y[a][b][i2]
            const T *gz = gtab + (kzc + j) * Q2;
#pragma unroll
            for (int bb = 0; bb < Q; ++bb) buf[L * RS + bb] = ya[bb];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            {
                const int a = L / Q, bb = L % Q;
                T y[Q];
#pragma unroll
                for (int i2 = 0; i2 < Q; ++i2) y[i2] = buf[(a * Q + i2) * RS + bb];
#pragma unroll
                for (int c = 0; c < Q; ++c) {
                    T s = T(0);
#pragma unroll
                    for (int i2 = 0; i2 < Q; ++i2) s += gz[c * Q + i2] * y[i2];
                    acc[c] += wj * s;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        e = ez;
    }
    // sum of the waves' partial sums, then the asymptotic part: Gaussians
    // with t >= t_a over R^3 from rho_B's polynomial
    __syncthreads();
    double *part = vsm;  // [JB][q^3]
#pragma unroll
    for (int c = 0; c < Q; ++c) part[w * Q3 + L * Q + c] = (double)acc[c];
    double *rB = part + JB * Q3, *d2 = rB + Q3, *l1 = d2 + Q2, *l2 = l1 + Q3;
    const double *rb = D.rho + (int64_t)vB * Q3;
    for (int t = tid; t < Q3; t += NT) rB[t] = rb[t];
    for (int t = tid; t < Q2; t += NT) d2[t] = D.d2[t];
    __syncthreads();
    const double lsc = 4.0 / (sB * sB);
    for (int o = tid; o < Q3; o += NT) {
        const int a = o / Q2, b = (o / Q) % Q, c = o % Q;
        double s = 0.0;
        for (int jx = 0; jx < Q; ++jx)
            s += d2[a * Q + jx] * rB[(jx * Q + b) * Q + c] + d2[b * Q + jx] * rB[(a * Q + jx) * Q + c] +
                 d2[c * Q + jx] * rB[(a * Q + b) * Q + jx];
        l1[o] = s * lsc;
    }
    __syncthreads();
    for (int o = tid; o < Q3; o += NT) {
        const int a = o / Q2, b = (o / Q) % Q, c = o % Q;
        double s = 0.0;
        for (int jx = 0; jx < Q; ++jx)
            s += d2[a * Q + jx] * l1[(jx * Q + b) * Q + c] + d2[b * Q + jx] * l1[(a * Q + jx) * Q + c] +
                 d2[c * Q + jx] * l1[(a * Q + b) * Q + jx];
        l2[o] = s * lsc;
    }
    __syncthreads();
    const double ta = D.tau_a / sB, ta2 = ta * ta;
    for (int o = tid; o < Q3; o += NT) {
        double near = 0.0;
#pragma unroll
        for (int g = 0; g < JB; ++g) near += part[g * Q3 + o];
        const double tail =
            2.0 * M_PI * (rB[o] / (2.0 * ta2) + l1[o] / (16.0 * ta2 * ta2) + l2[o] / (192.0 * ta2 * ta2 * ta2));
        D.unear[(int64_t)vB * Q3 + o] = near + tail;
    }
}

__global__ void __launch_bounds__(TPB) k_vol_finalize(const double *ufar, const double *unear, int64_t n, double *u,
                                                      double *fp, double *np)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    const double kap = 0.25 / M_PI;
    const double a = ufar[i] * kap, b = unear[i] * kap;
    if (u) u[i] = a + b;
    if (fp) fp[i] = a;
    if (np) np[i] = b;
}

inline unsigned vblk(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

template <typename K>
void vol_allow_lds(K kernel, size_t bytes)
{
    int dev = 0, lim = 0;
    DMK_HIP(hipGetDevice(&dev));
    DMK_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if ((size_t)lim < bytes) throw Error{DMK_ERR_UNSUPPORTED, "device LDS per workgroup too small for a volume stage"};
    DMK_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <typename T, int P, int Q>
void run_vol_t(Plan *Pl, const double *rho, double *u, double *fp, double *np, hipStream_t s)
{
    using LD = VolLds<P, Q>;
    static bool attrs = false;
    if (!attrs) {
        vol_allow_lds(k_vol_upward<T, P, Q>, LD::up(sizeof(T)));
        vol_allow_lds(k_vol_upward_q<T, P, Q>, LD::up(sizeof(T)));
        vol_allow_lds(k_vol_leaf<T, P, Q>, LD::leaf(sizeof(T)));
        vol_allow_lds(k_vol_near<T, Q, LD::JB>, LD::near(sizeof(T)));
        vol_allow_lds(k_vol_near<T, Q, LD::JB6>, LD::near(sizeof(T), LD::JB6));
        attrs = true;
    }
    VDev<T> D = make_vdev<T>(Pl);
    D.rho = rho;
    const auto &ll = Pl->ll;
    if (Pl->nfout && Pl->queued) {  // one queue-fed launch over all levels
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        const WorkQ q = upward_queue(Pl);
        reset_queue(q.head, 4 + Pl->nfout, s);
        static const unsigned nres = resident_blocks(k_vol_upward_q<T, P, Q>, TPB, LD::up(sizeof(T)));
        hipLaunchKernelGGL((k_vol_upward_q<T, P, Q>), dim3((unsigned)std::min<int64_t>(Pl->nfout, nres)), dim3(TPB),
                           LD::up(sizeof(T)), s, D, q);
    }
    for (int l = Pl->nlevels - 1; l >= 0 && !Pl->queued; --l) {
        const int64_t m = ll.fout_off[l + 1] - ll.fout_off[l];
        if (!m) continue;
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        hipLaunchKernelGGL((k_vol_upward<T, P, Q>), dim3((unsigned)m), dim3(TPB), LD::up(sizeof(T)), s, D,
                           Pl->l_fout + ll.fout_off[l]);
    }
    far_stages(Pl, s);
    {
        StageScope t(Pl, s, DMK_STAGE_LEAF);
        hipLaunchKernelGGL((k_vol_leaf<T, P, Q>), dim3((unsigned)Pl->nleaf), dim3(TPB), LD::leaf(sizeof(T)), s, D,
                           Pl->l_leaf);
    }
    {
        StageScope t(Pl, s, DMK_STAGE_RESIDUAL);
        VDev<double> D64 = make_vdev<double>(Pl);
        D64.rho = rho;
        const VolData &V = Pl->vol;
        const T *gtab = sizeof(T) == 8 ? (const T *)V.d_gtab : (const T *)V.f_gtab;
        if (V.split)  // 30 or 40 Gaussians per pair: ten waves share each staging of the sources
            hipLaunchKernelGGL((k_vol_near<T, Q, LD::JB6>), dim3((unsigned)Pl->nleaf), dim3(Q * Q * LD::JB6),
                               LD::near(sizeof(T), LD::JB6), s, D64, Pl->l_leaf, Pl->nl_off, Pl->nl_src, V.d_esrc,
                               V.d_pkey, gtab, V.d_gw);
        else
            hipLaunchKernelGGL((k_vol_near<T, Q, LD::JB>), dim3((unsigned)Pl->nleaf), dim3(Q * Q * LD::JB),
                               LD::near(sizeof(T)), s, D64, Pl->l_leaf, Pl->nl_off, Pl->nl_src, V.d_esrc, V.d_pkey,
                               gtab, V.d_gw);
    }
    {
        StageScope t(Pl, s, DMK_STAGE_FINALIZE);
        const int64_t n = Pl->vol.nleaf * Q * Q * Q;
        hipLaunchKernelGGL(k_vol_finalize, dim3(vblk(n)), dim3(TPB), 0, s, Pl->vol.ufar, Pl->vol.unear, n, u, fp, np);
    }
    DMK_HIP(hipGetLastError());
}

// PSWF split (tol 1e-6): the residual R_L(r) = (1 - Phi(r/s_L))/r of Sec. 3.7
// as Gaussians for the near field of Sec. 3.6.  In x = r/s_L,
//   (1 - Phi(x))/x = h(x) + (2/sqrt pi) int_{theta_1}^{tau} e^{-x^2 t^2} dt + erfc(tau x)/x,
//   h(x) = (erf(theta_1 x) - Phi(x))/x,  tau = t_a s_L:
// the integral is the log-t quadrature, erfc(tau x)/x the asymptotic part
// (Sec. 4.4), and h -- bounded, and zero to erfc(theta_1) beyond x = 1 -- is
// fitted here by n Gaussians e^{-x^2 t_i^2}, t_i geometric from 0.5 to 10,
// by least squares over 2200 equal steps of [0, 5.5] (node distances of a
// near pair stay below 3 sqrt 3 source sides), solved by Gram-Schmidt with
// reorthogonalisation.  fit = [t_i..., w_i...]; returns the largest error on
// the sample grid.
double vol_sog_fit(const Tables &tb, double theta1, int n, std::vector<double> &fit)
{
    const int m = 2200;
    fit.assign(2 * (size_t)n, 0.0);
    std::vector<double> t(n), xs(m), b(m), Q((size_t)n * m), R((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) t[i] = 0.5 * std::pow(20.0, (double)i / (n - 1));
    for (int j = 0; j < m; ++j) {
        const double x = 5.5 * j / (m - 1);
        xs[j] = x;
        b[j] = x == 0.0 ? 2.0 * theta1 / std::sqrt(M_PI) - tb.psi0 / tb.c0
                        : (std::erf(theta1 * x) - pswf_phi(tb, x)) / x;
    }
    for (int i = 0; i < n; ++i) {
        double *qi = &Q[(size_t)i * m];
        for (int j = 0; j < m; ++j) qi[j] = std::exp(-xs[j] * xs[j] * t[i] * t[i]);
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < i; ++k) {
                const double *qk = &Q[(size_t)k * m];
                double d = 0.0;
                for (int j = 0; j < m; ++j) d += qk[j] * qi[j];
                R[(size_t)k * n + i] += d;
                for (int j = 0; j < m; ++j) qi[j] -= d * qk[j];
            }
        double nr = 0.0;
        for (int j = 0; j < m; ++j) nr += qi[j] * qi[j];
        nr = std::sqrt(nr);
        if (!(nr > 0.0)) throw Error{DMK_ERR_STATE, "sum-of-Gaussians fit: singular basis"};
        R[(size_t)i * n + i] = nr;
        for (int j = 0; j < m; ++j) qi[j] /= nr;
    }
    std::vector<double> y(n), r(b);
    for (int i = 0; i < n; ++i) {  // y = Q^T b, one projection at a time
        const double *qi = &Q[(size_t)i * m];
        double d = 0.0;
        for (int j = 0; j < m; ++j) d += qi[j] * r[j];
        y[i] = d;
        for (int j = 0; j < m; ++j) r[j] -= d * qi[j];
    }
    for (int i = n - 1; i >= 0; --i) {
        double sum = y[i];
        for (int k = i + 1; k < n; ++k) sum -= R[(size_t)i * n + k] * fit[n + k];
        fit[n + i] = sum / R[(size_t)i * n + i];
    }
    double err = 0.0;
    for (int j = 0; j < m; ++j) {
        double sum = 0.0;
        for (int i = 0; i < n; ++i) sum += fit[n + i] * std::exp(-xs[j] * xs[j] * t[i] * t[i]);
        err = std::max(err, std::fabs(sum - b[j]));
    }
    for (int i = 0; i < n; ++i) fit[i] = t[i];
    return err;
}

// Gaussians of the near field of a pair whose target is 2^-k times the
// source side: Gauss-Legendre panels of width <= tpan_w in log t from
// sqL / s_T (Gaussian split: sqL = sqrt(log(1/eps)); PSWF split: theta_1)
// to tau_a / s_B; the PSWF split adds its nfit fitted Gaussians
int vol_npan(const VolData &V, int k)
{
    const double u0 = std::log(V.sqL), u1 = std::log(V.tau_a) + k * std::log(2.0);
    return std::max(1, (int)std::ceil((u1 - u0) / V.tpan_w - 1e-12));
}

// Plan-time pass over the gather lists: work counts for the model (merged
// children, shift pairs, near-field pairs and Gaussians) and the offset
// classes of the near field.  For a pair (source T, target B) that survives
// the pruning (box distance below s_T) each axis d has the class
// (k = L_B - L_T, delta = (c_B,d - c_T,d) / s_T): its 1-D factors for a unit
// source box depend on nothing else.
void vol_count_work(Plan *P, hipStream_t s)
{
    const int64_t nb = P->nbox, nl = P->nleaf;
    std::vector<uint8_t> fl(nb);
    std::vector<int32_t> c0(nb), col((size_t)nb * 27), lev(nb), leaf(nl), off(nl + 1);
    std::vector<double> cen((size_t)nb * 3);
    DMK_HIP(hipMemcpy(fl.data(), P->bflags, nb, hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(c0.data(), P->child0, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(col.data(), P->colleague, (size_t)nb * 27 * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(lev.data(), P->blevel, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(cen.data(), P->bcenter, (size_t)nb * 3 * sizeof(double), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(leaf.data(), P->l_leaf, nl * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(off.data(), P->nl_off, (nl + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    const int64_t ne = off[nl];
    std::vector<int32_t> src(std::max<int64_t>(ne, 1));
    DMK_HIP(hipMemcpy(src.data(), P->nl_src, (size_t)ne * sizeof(int32_t), hipMemcpyDeviceToHost));
    VolData &V = P->vol;
    V.n_merge = 0;
    P->n_shift_pairs = 0;
    for (int64_t b = 0; b < nb; ++b) {
        if (fl[b] & 2)
            for (int k = 0; k < 8; ++k)
                if (fl[c0[b] + k] & 2) V.n_merge++;
        if (fl[b] & 4)
            for (int k = 0; k < 27; ++k) {
                const int32_t j = col[(size_t)b * 27 + k];
                if (j >= 0 && (fl[j] & 2)) P->n_shift_pairs++;
            }
    }
    std::map<std::pair<int, uint64_t>, int32_t> cls;
    std::vector<int> ck;
    std::vector<double> cd;
    std::vector<int32_t> pkey((size_t)std::max<int64_t>(ne, 1) * 3, -1);
    V.n_pairs = V.n_gauss = 0;
    for (int64_t i = 0; i < nl; ++i) {
        const int32_t B = leaf[i];
        const double sB = std::ldexp(1.0, -lev[B]);
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            const int32_t T = src[e];
            const double sT = std::ldexp(1.0, -lev[T]);
            double gap2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double g = std::fabs(cen[3 * (size_t)B + d] - cen[3 * (size_t)T + d]) - 0.5 * (sB + sT);
                if (g > 0.0) gap2 += g * g;
            }
            if (gap2 >= sT * sT) continue;
            const int k = lev[B] - lev[T];
            for (int d = 0; d < 3; ++d) {
                const double delta = (cen[3 * (size_t)B + d] - cen[3 * (size_t)T + d]) / sT;  // exact (dyadic)
                uint64_t bits;
                std::memcpy(&bits, &delta, sizeof(bits));
                auto it = cls.find({k, bits});
                int32_t id;
                if (it == cls.end()) {
                    id = (int32_t)ck.size();
                    cls.emplace(std::make_pair(k, bits), id);
                    ck.push_back(k);
                    cd.push_back(delta);
                } else {
                    id = it->second;
                }
                pkey[3 * (size_t)e + d] = id;
            }
            V.n_pairs++;
            V.n_gauss += (int64_t)vol_npan(V, k) * V.tpan_gl + V.nfit;
        }
    }
    // order every target's entries by (z class, y class, x class), pruned
    // entries last, and mark the last entry of each (y, z) group and of each
    // z group: the near-field kernel sums x passes over a (y, z) group and
    // y passes over a z group before applying the next factor
    std::vector<int32_t> pk4((size_t)std::max<int64_t>(ne, 1) * 4, -1);
    {
        std::vector<int32_t> ord;
        for (int64_t i = 0; i < nl; ++i) {
            ord.clear();
            for (int32_t e = off[i]; e < off[i + 1]; ++e) ord.push_back(e);
            std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
                const int32_t *A = &pkey[3 * (size_t)a], *B = &pkey[3 * (size_t)b];
                const bool pa = A[0] < 0, pb = B[0] < 0;
                if (pa != pb) return pb;  // kept entries first
                if (pa) return false;
                if (A[2] != B[2]) return A[2] < B[2];
                if (A[1] != B[1]) return A[1] < B[1];
                return A[0] < B[0];
            });
            std::vector<int32_t> s2(ord.size());
            for (size_t r = 0; r < ord.size(); ++r) {
                const int32_t e = ord[r], d = off[i] + (int32_t)r;
                s2[r] = src[e];
                for (int k = 0; k < 3; ++k) pk4[4 * (size_t)d + k] = pkey[3 * (size_t)e + k];
            }
            for (size_t r = 0; r < ord.size(); ++r) {
                const int32_t d = off[i] + (int32_t)r;
                int32_t *K = &pk4[4 * (size_t)d];
                if (K[0] < 0) { K[3] = 0; continue; }
                const bool last = (r + 1 == ord.size()) || pk4[4 * (size_t)(d + 1)] < 0;
                const int32_t *N = last ? nullptr : &pk4[4 * (size_t)(d + 1)];
                const bool lz = last || N[2] != K[2];
                const bool ly = lz || N[1] != K[1];
                K[3] = (ly ? 1 : 0) | (lz ? 2 : 0);
            }
            for (size_t r = 0; r < ord.size(); ++r) src[off[i] + r] = s2[r];
        }
        // passes of the near-field kernel, times Gaussians: per z group an x
        // pass per entry, a y pass per (y, z) group and one z pass
        V.n_gauss_passes = 0;
        for (int64_t i = 0; i < nl; ++i) {
            int64_t npass = 0;
            for (int32_t e = off[i]; e < off[i + 1]; ++e) {
                const int32_t *K = &pk4[4 * (size_t)e];
                if (K[0] < 0) break;
                npass += 1 + (K[3] & 1) + ((K[3] >> 1) & 1);
                if (K[3] & 2) {
                    V.n_gauss_passes += npass * (vol_npan(V, ck[K[2]]) * V.tpan_gl + V.nfit);
                    npass = 0;
                }
            }
        }
        if (ne > 0)
            DMK_HIP(hipMemcpy(P->nl_src, src.data(), (size_t)ne * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    pkey.swap(pk4);
    // classes -> tables on the device
    const int64_t nk = (int64_t)ck.size();
    std::vector<int32_t> kng(std::max<int64_t>(nk, 1), 0), kk(std::max<int64_t>(nk, 1), 0);
    std::vector<int64_t> kbase(std::max<int64_t>(nk, 1), 0);
    int64_t ng = 0;
    for (int64_t c = 0; c < nk; ++c) {
        kng[c] = vol_npan(V, ck[c]) * V.tpan_gl + V.nfit;
        kk[c] = ck[c];
        kbase[c] = ng;
        ng += kng[c];
    }
    V.nkey = nk;
    V.ngauss_tab = ng;
    if (ng >= (int64_t(1) << 31) / 4) throw Error{DMK_ERR_STATE, "near-field tables too large"};
    // the near-field kernel reads table offsets, not class ids: each class
    // becomes the index of its first Gaussian, and the flags word carries the
    // entry's Gaussian count (its classes share one level difference) above bit 1
    for (int64_t e = 0; e < ne; ++e) {
        int32_t *K = &pkey[4 * (size_t)e];
        if (K[0] < 0) continue;
        const int32_t ngx = kng[K[0]];
        for (int d = 0; d < 3; ++d) K[d] = (int32_t)kbase[K[d]];
        K[3] |= ngx << 2;
    }
    const int q = V.q;
    auto upi = [&](const std::vector<int32_t> &h) {
        int32_t *d = (int32_t *)dalloc(P, h.size() * sizeof(int32_t));
        DMK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        return d;
    };
    V.d_pkey = upi(pkey);
    {  // volume leaf of each entry's source, in the sorted order
        std::vector<int32_t> b2v(nb), esrc(std::max<int64_t>(ne, 1), 0);
        DMK_HIP(hipMemcpy(b2v.data(), V.box2v, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < ne; ++e) esrc[e] = b2v[src[e]];
        V.d_esrc = (int32_t *)dalloc(P, esrc.size() * sizeof(int32_t));
        DMK_HIP(hipMemcpy(V.d_esrc, esrc.data(), esrc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    V.d_kng = upi(kng);
    int32_t *d_kk = upi(kk);
    V.d_kbase = (int64_t *)dalloc(P, kbase.size() * sizeof(int64_t));
    DMK_HIP(hipMemcpyAsync(V.d_kbase, kbase.data(), kbase.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    std::vector<double> cdp(cd);
    cdp.resize(std::max<int64_t>(nk, 1), 0.0);
    double *d_cd = (double *)dalloc(P, cdp.size() * sizeof(double));
    DMK_HIP(hipMemcpyAsync(d_cd, cdp.data(), cdp.size() * sizeof(double), hipMemcpyHostToDevice, s));
    V.d_gtab = (double *)dalloc(P, (size_t)std::max<int64_t>(ng, 1) * q * q * sizeof(double));
    V.d_gw = (double *)dalloc(P, (size_t)std::max<int64_t>(ng, 1) * sizeof(double));
    const int64_t rows = ng * q;
    if (rows > 0)
        hipLaunchKernelGGL(k_vol_gtab, dim3(vblk(rows)), dim3(TPB), 0, s, V.d_xq, V.d_tgl, V.d_tglw, V.d_egl,
                           V.d_eglw, V.tpan_gl, V.tpan_w, V.tau_a, V.sqL, q, nk, d_kk, d_cd, V.d_kng, V.d_kbase,
                           V.nfit, V.d_fit, rows, V.d_gtab, V.d_gw);
    if (P->precision == DMK_MIXED) {
        // the mixed path's near field multiplies in FP32
        const int64_t nt = std::max<int64_t>(ng, 1) * q * q;
        V.f_gtab = (float *)dalloc(P, (size_t)nt * sizeof(float));
        if (rows > 0) hipLaunchKernelGGL(k_vol_tof32, dim3(vblk(nt)), dim3(TPB), 0, s, V.d_gtab, V.f_gtab, nt);
    }
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

}  // namespace

// ------------------------------------------------------------------- plan
dmk_plan_t make_vol_plan(double tol, int32_t q, double rho_scale, int32_t min_level, int32_t max_level,
                         int32_t nfeat, const double *feat, dmk_density_fn density, void *ctx, const dmk_opts *opts,
                         void *stream)
{
    const bool pswf = (tol == 1e-6);  // PSWF split; tol 1e-3 takes the Gaussian split
    if (!(tol == 1e-3 || pswf))
        throw Error{DMK_ERR_UNSUPPORTED, "volume plans are built for tol = 1e-3 (Gaussian split) or 1e-6 (PSWF split)"};
    if (q != VQ) throw Error{DMK_ERR_UNSUPPORTED, "volume plans are built for q = 8"};
    if (!(rho_scale > 0) || !std::isfinite(rho_scale)) throw Error{DMK_ERR_ARG, "rho_scale must be positive"};
    if (min_level < 1 || max_level > 19 || min_level > max_level)
        throw Error{DMK_ERR_ARG, "need 1 <= min_level <= max_level <= 19"};
    if (!density) throw Error{DMK_ERR_ARG, "density is NULL"};
    if (nfeat < 0 || (nfeat > 0 && !feat)) throw Error{DMK_ERR_ARG, "bad feature list"};
    for (int32_t f = 0; f < nfeat; ++f)
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(feat[4 * (size_t)f + k]) || (k == 3 && !(feat[4 * (size_t)f + 3] > 0)))
                throw Error{DMK_ERR_ARG, "feature points need finite coordinates and h > 0"};
    dmk_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision != DMK_FP64 && o.precision != DMK_MIXED) throw Error{DMK_ERR_ARG, "unknown precision"};
    std::vector<Cell> tree = build_vol_tree(q, tol, rho_scale, min_level, max_level, nfeat, feat, density, ctx);
    const int q3 = q * q * q;
    const int64_t nleaf = (int64_t)tree.size();
    const int64_t n = nleaf * q3;
    if (n >= (int64_t(1) << 31)) throw Error{DMK_ERR_ARG, "more than 2^31 - 1 nodes"};
    Params prm;
    if (!params_for(1e-6, &prm, 3) || prm.p != 18 || prm.nf != 12)
        throw Error{DMK_ERR_STATE, "grid parameters p = 18, n_f = 12 unavailable"};
    auto *P = new Plan();
    try {
        hipStream_t s = (hipStream_t)stream;
        P->is_vol = true;
        P->fixed_root = true;
        P->dim = 3;
        P->kernel = DMK_LAPLACE;
        P->nprob = 1;
        P->poff = {0, n};
        P->pbits = 0;
        P->kb = 21;
        P->precision = o.precision;
        P->leaf_max = q3;
        P->max_depth = 20;
        if ((o.flags & DMK_FLAG_LEVEL_LAUNCHES) && (o.flags & DMK_FLAG_QUEUE_LAUNCHES))
            throw Error{DMK_ERR_ARG, "DMK_FLAG_LEVEL_LAUNCHES and DMK_FLAG_QUEUE_LAUNCHES exclude each other"};
        P->flags = o.flags & (DMK_FLAG_LEVEL_LAUNCHES | DMK_FLAG_QUEUE_LAUNCHES);
        P->queued = queue_schedule(3, P->flags);
        P->n = n;
        build_tables(prm, &P->tab, 3);
        if (!pswf) gauss_tables(&P->tab, tol);
        P->p = P->tab.p;
        P->nf = P->tab.nf;
        P->nw = P->tab.nw;
        VolData &V = P->vol;
        V.q = q;
        V.nleaf = nleaf;
        V.tau_a = 2.0 * std::pow(tol, -1.0 / 6.0);
        V.tpan_gl = 5;
        if (pswf) {
            // t-quadrature from theta_1 = 5 (erfc(5) = 1.5e-12 bounds h beyond
            // x = 1), 10 nodes per panel of width <= 1.4 in log t (one panel
            // up to t_a s_T = 20); 20 fitted Gaussians
            V.split = 1;
            V.sqL = 5.0;
            V.tpan_gl = 10;
            V.tpan_w = 1.4;
            V.nfit = 20;
            if (V.nfit % VolLds<18, VQ>::JB6 || V.tpan_gl % VolLds<18, VQ>::JB6)
                throw Error{DMK_ERR_STATE, "near-field Gaussians must fill whole passes"};
            V.fit_err = vol_sog_fit(P->tab, V.sqL, V.nfit, V.fit);
            if (!(V.fit_err < 2e-6)) throw Error{DMK_ERR_STATE, "sum-of-Gaussians fit of the residual failed"};
        } else {
            V.sqL = std::sqrt(std::log(1.0 / tol));
            V.tpan_w = 1.0;
        }
        V.level.resize(nleaf);
        V.ijk.resize(3 * nleaf);
        for (int64_t i = 0; i < nleaf; ++i) {
            V.level[i] = tree[i].l;
            for (int d = 0; d < 3; ++d) V.ijk[3 * i + d] = tree[i].c[d];
        }
        auto up64 = [&](const std::vector<double> &h) {
            double *d = (double *)dalloc(P, std::max<size_t>(h.size(), 1) * sizeof(double));
            DMK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
            return d;
        };
        auto up32i = [&](const std::vector<int32_t> &h) {
            int32_t *d = (int32_t *)dalloc(P, std::max<size_t>(h.size(), 1) * sizeof(int32_t));
            DMK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            return d;
        };
        P->d_poff = (int64_t *)dalloc(P, 2 * sizeof(int64_t));
        DMK_HIP(hipMemcpyAsync(P->d_poff, P->poff.data(), 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
        upload_tables(P, s);
        if (V.nfit) V.d_fit = up64(V.fit);
        V.d_level = up32i(V.level);
        V.d_ijk = up32i(V.ijk);
        std::vector<double> xq(q), bq(q);
        for (int a = 0; a < q; ++a) {
            xq[a] = std::cos(M_PI * (a + 0.5) / q);
            bq[a] = ((a & 1) ? -1.0 : 1.0) * std::sin((2 * a + 1) * M_PI / (2.0 * q));
        }
        V.d_xq = up64(xq);
        V.d_bq = up64(bq);
        // nodes -> point-code tree (root = unit cube, capacity q^3)
        double *pts = (double *)dalloc(P, (size_t)std::max<int64_t>(n, 1) * 3 * sizeof(double));
        hipLaunchKernelGGL(k_vol_nodes, dim3(vblk(n)), dim3(TPB), 0, s, V.d_level, V.d_ijk, V.d_xq, q, n, pts);
        build_tree(P, pts, s);
        build_lists(P, s);
        if (P->nleaf != nleaf) throw Error{DMK_ERR_STATE, "box tree does not reproduce the volume tree"};
        V.box2v = (int32_t *)dalloc(P, (size_t)P->nbox * sizeof(int32_t));
        DMK_HIP(hipMemsetAsync(V.box2v, 0xff, (size_t)P->nbox * sizeof(int32_t), s));
        unsigned long long *bad = (unsigned long long *)dalloc(P, sizeof(unsigned long long));
        DMK_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_vol_map, dim3(vblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, P->pstart, P->pcount,
                           P->perm, q3, V.box2v, bad);
        unsigned long long hbad = 0;
        DMK_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        if (hbad) throw Error{DMK_ERR_STATE, "box tree does not reproduce the volume tree"};
        // density -> parent proxy matrices V_s[a][j] = int ell_a((eta + s)/2) L_j(eta) d eta
        std::vector<double> gx, gw;
        gauss_legendre(18, gx, gw);
        const int p = P->p;
        std::vector<double> v1((size_t)2 * p * q, 0.0), la(p), lj(q);
        for (int sgn = 0; sgn < 2; ++sgn)
            for (size_t k = 0; k < gx.size(); ++k) {
                cheb_lagrange(p, 0.5 * (gx[k] + (sgn ? 1.0 : -1.0)), la.data());
                cheb_lagrange(q, gx[k], lj.data());
                for (int a = 0; a < p; ++a)
                    for (int j = 0; j < q; ++j) v1[((size_t)sgn * p + a) * q + j] += gw[k] * la[a] * lj[j];
            }
        V.d_v1 = up64(v1);
        {
            std::vector<float> f(v1.begin(), v1.end());
            V.f_v1 = (float *)dalloc(P, f.size() * sizeof(float));
            DMK_HIP(hipMemcpyAsync(V.f_v1, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, s));
            DMK_HIP(hipStreamSynchronize(s));
        }
        // second-derivative matrix of the leaf interpolant: D2 = D1 D1,
        // D1[i][j] = (w_j / w_i) / (x_i - x_j), D1[i][i] = -sum_{j != i} D1[i][j]
        std::vector<double> d1((size_t)q * q, 0.0), d2((size_t)q * q, 0.0);
        for (int i = 0; i < q; ++i) {
            double sd = 0.0;
            for (int j = 0; j < q; ++j) {
                if (j == i) continue;
                d1[i * q + j] = (bq[j] / bq[i]) / (xq[i] - xq[j]);
                sd += d1[i * q + j];
            }
            d1[i * q + i] = -sd;
        }
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < q; ++k) d2[i * q + j] += d1[i * q + k] * d1[k * q + j];
        V.d_d2 = up64(d2);
        std::vector<double> tx, tw, ex, ew;  // distinct buffers: the copies are asynchronous
        gauss_legendre(V.tpan_gl, tx, tw);
        V.d_tgl = up64(tx);
        V.d_tglw = up64(tw);
        gauss_legendre(32, ex, ew);
        V.d_egl = up64(ex);
        V.d_eglw = up64(ew);
        vol_count_work(P, s);
        alloc_workspace(P);
        V.ufar = (double *)dalloc(P, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
        V.unear = (double *)dalloc(P, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
        create_done_event(P);
        DMK_HIP(hipStreamSynchronize(s));
    } catch (...) {
        plan_release(P);
        throw;
    }
    return reinterpret_cast<dmk_plan_t>(P);
}

void vol_nodes(Plan *P, double *xyz, hipStream_t s)
{
    const int64_t n = P->n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_vol_nodes, dim3(vblk(n)), dim3(TPB), 0, s, P->vol.d_level, P->vol.d_ijk, P->vol.d_xq,
                       P->vol.q, n, xyz);
    DMK_HIP(hipGetLastError());
}

void run_vol_eval(Plan *P, const double *rho, double *u, double *far_part, double *near_part, hipStream_t s)
{
    if (P->vol.q != VQ || P->p != 18) throw Error{DMK_ERR_STATE, "volume plan with unexpected grid sizes"};
    if (P->precision == DMK_FP64)
        run_vol_t<double, 18, VQ>(P, rho, u, far_part, near_part, s);
    else
        run_vol_t<float, 18, VQ>(P, rho, u, far_part, near_part, s);
}

// Algorithmic work of one volume eval (FP64): flops of the separable
// contractions, bytes that must cross HBM once.
//   upward    2 (q^3 p + q^2 p^2 + q p^3) per leaf (density -> parent grid),
//             6 p^4 per merged child; density read once, proxies written once
//   far       as the point code (proxy->PW, translation, PW->grid, root)
//   leaf      2 (p^3 q + p^2 q^2 + p q^3) per leaf; anchor grid read, q^3 written
//   residual  2 q^4 per pass and Gaussian (one q x q mode product over a
//             q^3 block): an x pass per kept pair, a y pass per (y, z) group
//             and a z pass per z group of a target's sorted gather list; and
//             12 q^4 per leaf (two Laplacians); density read, near part written
void vol_stage_work(const Plan *P, double *F, double *Bt)
{
    const Tables &t = P->tab;
    const double el = (P->precision == DMK_FP64) ? 8.0 : 4.0, p = t.p, n = t.nn, nh = t.nh, q = P->vol.q;
    const double p3 = p * p * p, p4 = p3 * p, q3 = q * q * q, q4 = q3 * q;
    const double NL = (double)P->vol.nleaf, N = (double)P->n;
    for (int i = 0; i < DMK_NSTAGES; ++i) F[i] = Bt[i] = 0.0;
    const double pwflops = 4 * nh * p3 + 8 * nh * n * p * p + 8 * nh * n * n * p;
    const double pwbytes = 2 * el * nh * n * n;
    F[DMK_STAGE_UPWARD] = 2 * (q3 * p + q * q * p * p + q * p3) * NL + 6 * p4 * P->vol.n_merge;
    Bt[DMK_STAGE_UPWARD] = 8 * q3 * NL + el * p3 * (P->vol.n_merge + P->nfout);
    const double nw = t.nwn, nwh = t.nwh;
    F[DMK_STAGE_ROOT] = 2 * (4 * nwh * p3 + 8 * nwh * nw * p * p + 8 * nwh * nw * nw * p);
    Bt[DMK_STAGE_ROOT] = 16 * p3;
    F[DMK_STAGE_PROXY2PW] = pwflops * P->nfout;
    Bt[DMK_STAGE_PROXY2PW] = (el * p3 + pwbytes) * P->nfout;
    F[DMK_STAGE_PWSHIFT] = 8 * nh * n * n * P->n_shift_pairs;
    Bt[DMK_STAGE_PWSHIFT] = pwbytes * (P->nfout + P->nfin);
    F[DMK_STAGE_PW2GRID] = pwflops * P->nfin + 6 * p4 * std::max<int64_t>(P->nanc - 1, 0);
    Bt[DMK_STAGE_PW2GRID] = pwbytes * P->nfin + 2 * el * p3 * P->nanc;
    F[DMK_STAGE_LEAF] = 2 * (p3 * q + p * p * q * q + p * q3) * NL;
    Bt[DMK_STAGE_LEAF] = el * p3 * P->nanc + 8 * N;
    F[DMK_STAGE_RESIDUAL] = 2 * q4 * (double)P->vol.n_gauss_passes + 12 * q4 * NL;
    Bt[DMK_STAGE_RESIDUAL] = 16 * N;
    Bt[DMK_STAGE_FINALIZE] = 24 * N;
}

}  // namespace dmk
