// Steps 2-5 of the discrete DMK algorithm (Sec. 3.5) on gfx950.
//
// Every stage is written once as a template over the arithmetic type T
// (double for the FP64 path, float for the mixed path), the Chebyshev order
// P and the plane-wave half width NF.  The tensor-product transforms are
// sequences of small dense contractions (Lemmas 2.1/2.2, eqs.
// outgoingexpansion2/incomingexpansion2); the plane-wave transforms, the
// local values and the leaf evaluation run them on the matrix cores
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64), the upward pass as
// register-tiled products on the vector ALUs.
//
//   k_upward_q   proxy charges of each F_out box, all levels in one launch
//                fed by a device work queue (k_upward: one level): F_out
//                children are merged with the child->parent anterpolation
//                matrices (Lemma 2.1); the points of all other children are
//                anterpolated straight onto the parent's grid (Def. 2.1,
//                exact by Lemma 2.1).
//   k_root_stage windowed kernel W_0 on the root grid (FP64 always).
//   k_proxy2pw_mfma  outgoing plane waves Phi_l(B) of F_out boxes.
//   k_pwshift    incoming plane waves Psi_l(B) from the F_out colleagues
//                (diagonal translation; with h_l s_l = 2 pi/3 the phases
//                are cube roots of unity).
//   k_local_mfma_q  local values of the anchor boxes (the root and the
//                boxes with F_in), all levels from a work queue
//                (k_local_mfma: one level): interpolation of the nearest
//                anchor ancestor's polynomial to the box's grid (Lemma 2.2)
//                plus the box's own incoming plane waves on that grid.
//   k_leaf_mfma  far potential at the targets of each leaf, read from its
//                anchor's polynomial (a box without F_in adds nothing of its
//                own, so its polynomial is its anchor's, restricted).
//   k_residual   residual-kernel sums in gather form with the r = 0 self
//                correction (Steps 4-5).
//   k_finalize   scaling by 1/(4 pi S), scatter to input order.
//
// HBM layout: sorted points SoA FP64; per-box p^3 arrays (x index slowest);
// plane waves planar (all real parts, then all imaginary parts), index
// [m1][m3][m2] with m1, m2 in -nf..nf and m3 in 0..nf (Hermitian half).
#include <algorithm>
#include <cmath>

#include "dmk_internal.h"
#include "lagrange.h"
#include "queue.h"
#include "tiles.h"

namespace dmk {

namespace {

// ------------------------------------------------------------ device view
// elements per plane-wave set (real or imaginary part of one box): the
// nh * nn * nn modes of the half spectrum, padded to a multiple of 64 so that
// every set starts 256-byte aligned
static inline int64_t pw_stride(const Tables &t) { return ((int64_t)t.nh * t.nn * t.nn + 63) / 64 * 64; }

template <typename T>
struct Dev {
    int p, nf, nn, nh, nw, nwn, nwh, gdeg;
    const double *X, *Y, *Z, *qs;
    const int32_t *pstart, *pcount, *child0, *parent, *col, *proxy_slot, *local_slot, *psi_slot, *blevel,
        *anchor;
    const uint8_t *bflags;
    const uint8_t *anc_read;  // per anchor slot: its values are read by a finer anchor
    const double *bcenter;
    const T *c2p, *epw, *wd0, *gcheb, *gmono, *xcheb, *bary;  // tables in T
    const double *ew64, *ww64, *xcheb64, *bary64;     // FP64 tables
    T *proxy, *local, *phi, *psi, *w0vals;
    double *ufar, *ures, *rootscratch;
    int64_t pwstride;  // elements per plane-wave set: nh * nn * nn modes, padded to a multiple of 64
    // Yukawa e^{-lambda r}/r (null ywd for 1/r): per-level D_l weights, the
    // mollified kernels' series per level, M_l(0), lambda in root units
    const T *ywd, *ycheb;
    const double *yself;
    int64_t ywd_stride;
    double ylam;
    int ydeg, ynlev;
    int wshift;  // level-l weights are 2^(wshift l) times level 0's: 1 for 1/r, 2 for 1/r^2
    // batches of independent problems: root scratch per problem, and the
    // most points a root leaf holds (the scratch's Lagrange-row region)
    int64_t root_stride;
    int root_npmax;
    // targets (the sources' arrays unless the plan has separate target sets):
    // tree-order coordinates and per-box ranges; X, Y, Z, pstart, pcount and
    // qs above are the sources
    const double *Xt, *Yt, *Zt;
    const int32_t *tstart, *tcount;
};

// ------------------------------------------------------------------ upward
// x slabs of a child's proxy grid per round of the child -> parent mode
// products: all p, except FP64 at p = 18, whose two p^3 work buffers (93 KB)
// leave room for one block per CU, against two with 2 x 6 p^2 (at p = 15 and
// 9 the registers, not the LDS, set the occupancy)
template <typename T, int P> constexpr int up_slabs() { return sizeof(T) == 8 && P == 18 ? 6 : P; }

// the upward kernel's work area (values): two buffers of up_slabs x p^2
template <typename T, int P> constexpr int up_work() { return 2 * up_slabs<T, P>() * P * P; }

// points per anterpolation chunk: three Lagrange rows per point in the work area
template <typename T, int P> constexpr int up_chunk()
{
    return up_work<T, P>() / (3 * P) < 128 ? up_work<T, P>() / (3 * P) : 128;
}

// COH: the box's children were computed by the same launch (queue-fed)
template <typename T, int P, bool COH>
__device__ __forceinline__ void upward_box(const Dev<T> &D, const int32_t Pb)
{
    constexpr int P2 = P * P, P3 = P2 * P, RM = Tiles<P>::RM, RN = Tiles<P>::RN;
    constexpr int ZM = Tiles<P>::ZM, ZN = Tiles<P>::ZN, CH = up_chunk<T, P>(), GS = up_slabs<T, P>();
    constexpr int MT = (P + RM - 1) / RM, NT = (P2 + RN - 1) / RN;  // tile grid of the p x p^2 accumulator
    extern __shared__ __align__(16) unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    T *Am = sm;              // 2 p^2 child->parent matrices
    T *xc = Am + 2 * P2;     // nodes
    T *bw = xc + P;          // barycentric weights
    T *w0 = bw + P;          // work area of up_work values
    for (int t = threadIdx.x; t < 2 * P2; t += TPB) Am[t] = D.c2p[t];
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    T acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = T(0);
    const double *cP = D.bcenter + 3 * (int64_t)Pb;
    const double sc = 2.0 / box_side(D.blevel[Pb]);
    // the leaf children's point ranges, concatenated (their anterpolation does
    // not depend on the child: every point goes onto the parent's grid)
    __shared__ int64_t rlo[8];
    __shared__ int roff[9];
    int nr = 0, npts = 0;
    if (threadIdx.x == 0) roff[0] = 0;
    __syncthreads();
    for (int k = 0; k < 8; ++k) {
        const int32_t C = D.child0[Pb] + k;
        const int cnt = D.pcount[C];
        if (cnt == 0) continue;
        if (D.bflags[C] & 2) {
            // c2p: three mode products with A_sigma (sigma from the child's
            // position), GS x slabs (i0) at a time
            const T *src = D.proxy + (int64_t)D.proxy_slot[C] * P3;
            T *t1 = w0, *t2 = w0 + GS * P2;
            const T *Ax = Am + ((k >> 2) & 1) * P2, *Ay = Am + ((k >> 1) & 1) * P2, *Az = Am + (k & 1) * P2;
            for (int i00 = 0; i00 < P; i00 += GS) {
                const int g = min(GS, P - i00);
                __syncthreads();
                copy_to_lds<COH, TPB>(t2, src + i00 * P2, g * P2);
                __syncthreads();
                // z: t1[(i0 i1)][a2] = sum_i2 t2[(i0 i1)][i2] Az[a2][i2]
                gemm<T, ZM, ZN, false>(1, g * P, P, P, t2, 0, P, 1, Az, 0, 1, P, t1, 0, P, 1);
                __syncthreads();
                // y: t2[i0][a1][a2] = sum_i1 Ay[a1][i1] t1[i0][i1][a2]
                gemm<T, ZM, ZN, false>(g, P, P, P, Ay, 0, P, 1, t1, P2, P, 1, t2, P2, P, 1);
                __syncthreads();
                // x: acc[a0][r] += sum_i0 Ax[a0][i0] t2[i0][r] over the round's slabs
                gemm_regs<T, RM, RN>(P, P2, g, Ax + i00, P, 1, t2, P2, 1, acc);
            }
        } else {
            if (threadIdx.x == 0) {
                rlo[nr] = D.pstart[C];
                roff[nr + 1] = npts + cnt;
            }
            npts += cnt;
            ++nr;
        }
    }
    // anterpolate the leaf children's points onto the parent grid:
    // rho[a0][(a1 a2)] += sum_pt Lx[pt][a0] Ly[pt][a1] (Lz[pt][a2] q[pt]),
    // the product Ly Lz q formed per k step for the thread's columns
    if (npts > 0) {
        static_assert(NT % P == 0, "column tiles step whole rows of the p x p block");
        T *Lx = w0, *Ly = Lx + CH * P, *Lzq = Ly + CH * P;
        const int t = threadIdx.x;
        const bool own = t < MT * NT;
        const int mt = own ? t / NT : 0, nt = own ? t % NT : 0;
        // column n = nt + j NT of the thread is (a1, a2) = (nt / P + j NT / P, nt % P)
        const int c10 = nt / P, c2 = nt % P;
        for (int base = 0; base < npts; base += CH) {
            const int m = min(CH, npts - base);
            __syncthreads();
            for (int u = threadIdx.x; u < 3 * m; u += TPB) {
                const int pt = u / 3, d = u % 3;
                const int v = base + pt;
                int r = 0;
                while (v >= roff[r + 1]) ++r;
                const int64_t i = rlo[r] + (v - roff[r]);
                const double x = (d == 0) ? D.X[i] : (d == 1) ? D.Y[i] : D.Z[i];
                T row[P];
                lagrange_row<T>(P, xc, bw, (T)((x - cP[d]) * sc), row);
                const T f = (d == 2) ? (T)D.qs[i] : T(1);
                T *dst = (d == 0 ? Lx : d == 1 ? Ly : Lzq) + pt * P;
#pragma unroll
                for (int a = 0; a < P; ++a) dst[a] = row[a] * f;
            }
            __syncthreads();
            if (own) {
                // partial sums over runs of up to 32 points, then added to acc
                // (shorter running sums: these charges cancel heavily)
                for (int k0 = 0; k0 < m; k0 += 32) {
                    T part[RM][RN];
#pragma unroll
                    for (int i = 0; i < RM; ++i)
#pragma unroll
                        for (int j = 0; j < RN; ++j) part[i][j] = T(0);
                    const int k1 = min(m, k0 + 32);
                    for (int k = k0; k < k1; ++k) {
                        T a[RM], bb[RN];
#pragma unroll
                        for (int i = 0; i < RM; ++i) {
                            const int mm = mt + i * MT;
                            a[i] = (mm < P) ? Lx[k * P + mm] : T(0);
                        }
                        const T lz = Lzq[k * P + c2];
#pragma unroll
                        for (int j = 0; j < RN; ++j) {
                            const int c1 = c10 + j * (NT / P);
                            bb[j] = (c1 < P) ? Ly[k * P + c1] * lz : T(0);
                        }
#pragma unroll
                        for (int i = 0; i < RM; ++i)
#pragma unroll
                            for (int j = 0; j < RN; ++j) part[i][j] += a[i] * bb[j];
                    }
#pragma unroll
                    for (int i = 0; i < RM; ++i)
#pragma unroll
                        for (int j = 0; j < RN; ++j) acc[i][j] += part[i][j];
                }
            }
        }
    }
    store_tiles<T, P, COH>(acc, D.proxy + (int64_t)D.proxy_slot[Pb] * P3);
}

// one level's F_out boxes, one workgroup per box
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_upward(Dev<T> D, const int32_t *list)
{
    upward_box<T, P, false>(D, list[blockIdx.x]);
}

// the F_out boxes of every level, finest first, from the work queue: a box
// waits for its F_out children
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_upward_q(Dev<T> D, WorkQ q)
{
    queue_loop(
        q,
        [&](int32_t Pb) {
            if (threadIdx.x < 8) {
                const int32_t C = D.child0[Pb] + threadIdx.x;
                if (D.pcount[C] > 0 && (D.bflags[C] & 2)) wait_done(q, C);
            }
        },
        [&](int32_t Pb) { upward_box<T, P, true>(D, Pb); });
}

// ------------------------------------------------ diagonal translation
// Incoming plane waves of the children of one parent (a sibling group).  The
// colleagues of the 8 children lie in the 4x4x4 block of boxes around them;
// child t sits at cell t + (1,1,1).  With delta = (c_S - c_B)/s_l the
// translation factor exp(i h m.(c_B - c_S)) = w^{-(m.delta)}, w = e^{2 pi i/3}
// (h_l s_l = 2 pi/3), factors per axis, so the 27-term sum of each child runs
// as three passes of 3-term sums (z, then y, then x) shared by the siblings:
// 64 loads per mode for 8 boxes instead of up to 27 per box.  Each 3-term sum
// is a x + y + conj(a) z with a = w^{-m_k} for the axis, which takes 8
// operations in the form below (a complex multiply alone takes 6).
//
// Each source is read by every group that has it in its 4x4x4 block (6.6
// groups on average for clustered points), mostly from L2.  The stage waits
// on loads: a wave's loads complete in order, so a batch waits for its
// slowest, often an HBM miss, and what keeps the memory system busy is the
// number of resident waves rather than the size of each wave's batches.  So
// the kernel keeps its registers few (8 waves per SIMD in FP32, 5 in FP64)
// and its batches small (one or two rows of 4 sources), does no arithmetic
// beyond those sums (one thread per mode), keeps the box lists and the tests
// on them in scalar registers (they are the same for the whole workgroup,
// read through the scalar cache), addresses its loads from a scalar base,
// and loads nothing for absent sources or empty rows and slabs.
//
// A block covers TPB consecutive modes of one group.  Blocks are dealt out
// so that each XCD gets a contiguous range of groups, and within it the
// blocks run chunk by chunk over that range: neighbouring groups share most
// of their sources, and a source's chunk is then read again by the next few
// groups while it is still in that XCD's L2.
template <typename T>
struct Cx { T r, i; };

// a x + y + conj(a) z, a = (c, s)
template <typename T>
__device__ __forceinline__ Cx<T> sum3(T c, T s, Cx<T> x, Cx<T> y, Cx<T> z)
{
    const T u = x.r + z.r, v = x.i - z.i, p = x.i + z.i, q = x.r - z.r;
    return {fma(c, u, fma(-s, v, y.r)), fma(c, p, fma(s, q, y.i))};
}

// w^{-k} = (cos, sin) for any integer k
template <typename T>
__device__ __forceinline__ void root3(int k, T &c, T &s)
{
    k %= 3;
    if (k < 0) k += 3;
    const T s3 = T(0.86602540378443864676);
    c = k == 0 ? T(1) : T(-0.5);
    s = k == 0 ? T(0) : (k == 1 ? -s3 : s3);
}

// the value at byte offset `off` (per thread) of the `bytes` bytes at a
// workgroup-uniform base, through a buffer descriptor built in scalar
// registers (no per-thread address arithmetic; 0x20000: 32-bit data format)
template <typename T>
__device__ __forceinline__ T ld_buf(const T *base, uint32_t bytes, uint32_t off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), (short)0, (int)bytes, 0x00020000);
    T v;
    if constexpr (sizeof(T) == 4) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
        __builtin_memcpy(&v, &u, sizeof(T));
    } else {
        static_assert(sizeof(T) == 8, "float or double");
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        __builtin_memcpy(&v, &u, sizeof(T));
    }
    return v;
}

// RB source rows (4 RB boxes) are loaded at a time, all issued before the
// first is used.
template <typename T, int RB>
__global__ void __launch_bounds__(TPB, sizeof(T) == 4 ? 8 : 5)
    k_pwshift(Dev<T> D, const int32_t *oct_dst, const int32_t *oct_src, const int32_t *oct_level, int64_t noct,
              int nchunk)
{
    static_assert(4 % RB == 0, "rows per batch");
    // grid = 8 * per * nchunk; blocks go to the XCDs round-robin
    const int64_t per = (noct + 7) / 8;  // groups per XCD
    const int64_t Lb = blockIdx.x / 8;
    const int chunk = (int)(Lb / per);
    const int64_t o = (int64_t)(blockIdx.x % 8) * per + Lb % per;
    const int nn = D.nn, nh = D.nh, nf = D.nf;
    const int nmode = nh * nn * nn;
    const int e = chunk * TPB + (int)threadIdx.x;
    if (o >= noct || e >= nmode) return;
    const int32_t *src = oct_src + o * 64, *dst = oct_dst + o * 8;
    const int64_t nm = D.pwstride;
    const uint32_t eb = (uint32_t)e * sizeof(T);         // byte offset of this thread's mode in a set
    const uint32_t hbytes = (uint32_t)(nm * sizeof(T));  // the real part, then the imaginary part
    // per-axis factors a = w^{-m}; e = (m1 * nh + m3) * nn + m2
    T xc, xs, yc, ys, zc, zs;
    root3<T>(-(e / (nn * nh) - nf), xc, xs);
    root3<T>(-(e % nn - nf), yc, ys);
    root3<T>(-((e / nn) % nh), zc, zs);
    const Cx<T> zero = {T(0), T(0)};
    // acc[tx][ty][tz]: the x pass, accumulated slab by slab (slab gx enters
    // tx = gx with factor a, tx = gx - 1 with 1 and tx = gx - 2 with conj(a))
    Cx<T> acc[2][2][2];
#pragma unroll
    for (int tx = 0; tx < 2; ++tx)
#pragma unroll
        for (int ty = 0; ty < 2; ++ty)
#pragma unroll
            for (int tz = 0; tz < 2; ++tz) acc[tx][ty][tz] = zero;
#pragma unroll
    for (int gx = 0; gx < 4; ++gx) {
        // the slab is empty when all 16 of its entries are negative
        int32_t all = -1;
#pragma unroll
        for (int k = 0; k < 16; ++k) all &= src[gx * 16 + k];
        if (all < 0) continue;
        Cx<T> Z[4][2];  // z pass of each row: Z[gy][tz]
#pragma unroll
        for (int gy0 = 0; gy0 < 4; gy0 += RB) {
            Cx<T> f[RB][4];
            bool rempty[RB];  // rows with no source are not loaded
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                const int32_t *rw = src + (gx * 4 + gy0 + a) * 4;
                rempty[a] = (rw[0] & rw[1] & rw[2] & rw[3]) < 0;
                if (rempty[a]) continue;
#pragma unroll
                for (int gz = 0; gz < 4; ++gz) {
                    const int32_t sl = rw[gz];
                    f[a][gz] = zero;
                    if (sl < 0) continue;
                    const T *q = D.phi + 2 * (int64_t)sl * nm;
                    f[a][gz] = {ld_buf(q, 2 * hbytes, eb), ld_buf(q, 2 * hbytes, eb + hbytes)};
                }
            }
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                if (rempty[a]) {
                    Z[gy0 + a][0] = zero;
                    Z[gy0 + a][1] = zero;
                    continue;
                }
                Z[gy0 + a][0] = sum3(zc, zs, f[a][0], f[a][1], f[a][2]);
                Z[gy0 + a][1] = sum3(zc, zs, f[a][1], f[a][2], f[a][3]);
            }
        }
#pragma unroll
        for (int ty = 0; ty < 2; ++ty)
#pragma unroll
            for (int tz = 0; tz < 2; ++tz) {
                const Cx<T> Y = sum3(yc, ys, Z[ty][tz], Z[ty + 1][tz], Z[ty + 2][tz]);
                const Cx<T> aY = {xc * Y.r - xs * Y.i, xc * Y.i + xs * Y.r};  // a Y
                const Cx<T> cY = {xc * Y.r + xs * Y.i, xc * Y.i - xs * Y.r};  // conj(a) Y
                if (gx <= 1) {
                    acc[gx][ty][tz].r += aY.r;
                    acc[gx][ty][tz].i += aY.i;
                }
                if (gx >= 1 && gx <= 2) {
                    acc[gx - 1][ty][tz].r += Y.r;
                    acc[gx - 1][ty][tz].i += Y.i;
                }
                if (gx >= 2) {
                    acc[gx - 2][ty][tz].r += cY.r;
                    acc[gx - 2][ty][tz].i += cY.i;
                }
            }
    }
    // the level's weight, and the stores
    // 1/r: w_l = 2^l w_0, 1/r^2: 4^l w_0 (scale invariance); Yukawa: the level's own table
    const T scale = D.ywd ? T(1) : (T)ldexp(1.0, D.wshift * oct_level[o]);
    const T *wt = D.ywd ? D.ywd + (int64_t)oct_level[o] * D.ywd_stride : D.wd0;
    const T w = wt[e] * scale;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int32_t d = dst[t];
        if (d < 0) continue;
        const Cx<T> v = acc[t >> 2][(t >> 1) & 1][t & 1];
        char *out = reinterpret_cast<char *>(D.psi + 2 * (int64_t)d * nm) + eb;
        // streaming stores: Psi is read again only by the local stage, long
        // after, so it should not displace the sources held in L2
        __builtin_nontemporal_store(v.r * w, reinterpret_cast<T *>(out));
        __builtin_nontemporal_store(v.i * w, reinterpret_cast<T *>(out + hbytes));
    }
}

// ------------------------------------------ local values on matrix cores
// FP32 path of the local stage on MFMA (v_mfma_f32_16x16x4f32).  Every step
// is a mode product Y(x, a) = sum_k X(x, k) B(k, a) with x running over the
// two untouched indices (up to 325 rows) and a over the new one: waves take
// 16-row slabs of x, 16-column tiles of a, and 4-deep steps of k; lane l
// supplies X(x0 + l%16, k0 + l/16) and B(k0 + l/16, a0 + l%16) and receives
// Y(x0 + 4(l/16) + i, a0 + l%16), i < 4.  B (the small interpolation and
// plane-wave matrices) is loaded once into registers per tile.
//   interpolation from the anchor (Lemma 2.2): contract x, then y, then z;
//   plane waves -> grid (eq. incomingexpansion2): contract m1 (complex),
//   then m2 (complex), then m3 with the real part and the half-spectrum
//   weights; the last step lands in the same (x = (j1 j2), a = j3)
//   fragments as the interpolation's last step, so both stay in registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int NWAVE = TPB / 64;

// one 16x16x4 matrix-core product in T: v_mfma_f32_16x16x4f32 or
// v_mfma_f64_16x16x4f64.  Both take A(l%16, l/16) and B(l/16, l%16) from
// lane l; they differ in where the 16x16 result lands: item q of lane l is
// D(4(l/16) + q, l%16) in FP32 and D(l/16 + 4q, l%16) in FP64 (RB, RS)
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    using v4 = f32x4;
    static constexpr int RB = 4, RS = 1;  // result item q of lane l: row RB (l / 16) + RS q
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    using v4 = f64x4;
    static constexpr int RB = 1, RS = 4;
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <typename T>
using v4_t = typename Mfma<T>::v4;

constexpr int LOCAL_NT = 512;  // threads per block of the local stage (more waves hide MFMA latency)

template <typename T, int P, int NF>
struct LocalMfma {
    static constexpr int P2 = P * P, P3 = P2 * P, NN = 2 * NF + 1, NH = NF + 1, NM = NH * NN;
    static constexpr int NSL = (P2 + 15) / 16;              // slabs of the p^2 x p outputs
    static constexpr int NWV = LOCAL_NT / 64, NT = LOCAL_NT;  // waves and threads per block
    static constexpr int NSW = (NSL + NWV - 1) / NWV;       // slabs per wave
    static constexpr int G = 16 / (P % 16 == 0 ? 16 : (P % 8 == 0 ? 8 : (P % 4 == 0 ? 4 : (P % 2 == 0 ? 2 : 1))));
    static constexpr int KP = 2 * NH;                        // m3 real parts, then imaginary parts
    static constexpr int TAB = 2 * NN * P + KP * P + 3 * P2 + 2 * P;
    static constexpr int WORK_P2C = 2 * P3;
    static constexpr int WORK_PW = 2 * P * NM + G * P * KP;
    static constexpr int WORK = WORK_P2C > WORK_PW ? WORK_P2C : WORK_PW;
    static size_t lds() { return sizeof(T) * (TAB + WORK); }
};

// Column split of a p-wide new index: 16-column MFMA tiles, and a remainder
// of at most 4 columns (p = 18: columns 16, 17) done on the vector ALUs.  A
// padded tile would spend a whole MFMA chain on those 2 columns (44 % of the
// matrix-core work at p = 18); on the VALU they cost 2 FMAs per k step.
template <int P>
struct ColSplit {
    static constexpr int REM = P % 16;
    static constexpr int NATM = P / 16 + (REM > 4 ? 1 : 0);  // MFMA column tiles
    static constexpr int NREM = REM > 4 ? 0 : REM;           // remainder columns on the VALU
    static constexpr int NRA = NREM > 0 ? NREM : 1;          // array extent for them
};

// sum over the four k quarters of a fragment (lanes r16, r16+16, r16+32, r16+48)
template <typename T>
__device__ inline T kq_sum(T v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// real mode product into registers: acc[i][t] += sum_k X(x, k) B(k, a) for the
// wave's slabs i (slab w + NWV i) and tiles t; Bt[k * P + a].  The remainder
// columns a = 16 NATM + j go to accr[i][j] for row 16 sl + r16 (the same value
// in the four lanes of a row).
template <int NWV, int P, int NX, int NK, int NSW, typename XF, typename T>
__device__ inline void mma_real_acc(XF X, const T *Bt, v4_t<T> (&acc)[NSW][ColSplit<P>::NATM],
                                    T (&accr)[NSW][ColSplit<P>::NRA])
{
    constexpr int NATM = ColSplit<P>::NATM, NREM = ColSplit<P>::NREM, NRA = ColSplit<P>::NRA;
    constexpr int NKS = (NK + 3) / 4, NSL = (NX + 15) / 16;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    T breg[NATM][NKS], brem[NRA][NKS];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kq;
#pragma unroll
        for (int t = 0; t < NATM; ++t) {
            const int a = 16 * t + r16;
            breg[t][s] = (k < NK && a < P) ? Bt[k * P + a] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NREM; ++j) brem[j][s] = (k < NK) ? Bt[k * P + 16 * NATM + j] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int sl = w + NWV * i;
        if (sl >= NSL) break;  // uniform in the wave
        const int xa = 16 * sl + r16;
        T pr[NRA];
#pragma unroll
        for (int j = 0; j < NRA; ++j) pr[j] = T(0);
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kq;
            const T av = (xa < NX && k < NK) ? X(xa, k) : T(0);
#pragma unroll
            for (int t = 0; t < NATM; ++t)
                acc[i][t] = Mfma<T>::mma(av, breg[t][s], acc[i][t]);
#pragma unroll
            for (int j = 0; j < NREM; ++j) pr[j] += av * brem[j][s];
        }
#pragma unroll
        for (int j = 0; j < NREM; ++j) accr[i][j] += kq_sum(pr[j]);
    }
}

// real mode product with the result stored: Y(x, a) -> store(x, a, v)
template <int NWV, int P, int NX, int NK, typename XF, typename SF, typename T>
__device__ inline void mma_real_store(XF X, const T *Bt, SF store)
{
    constexpr int NATM = ColSplit<P>::NATM, NREM = ColSplit<P>::NREM, NRA = ColSplit<P>::NRA;
    constexpr int NKS = (NK + 3) / 4, NSL = (NX + 15) / 16;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    T breg[NATM][NKS], brem[NRA][NKS];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kq;
#pragma unroll
        for (int t = 0; t < NATM; ++t) {
            const int a = 16 * t + r16;
            breg[t][s] = (k < NK && a < P) ? Bt[k * P + a] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NREM; ++j) brem[j][s] = (k < NK) ? Bt[k * P + 16 * NATM + j] : T(0);
    }
    for (int sl = w; sl < NSL; sl += NWV) {
        const int xa = 16 * sl + r16;
        v4_t<T> acc[NATM];
        T pr[NRA];
#pragma unroll
        for (int t = 0; t < NATM; ++t) acc[t] = v4_t<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < NRA; ++j) pr[j] = T(0);
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kq;
            const T av = (xa < NX && k < NK) ? X(xa, k) : T(0);
#pragma unroll
            for (int t = 0; t < NATM; ++t) acc[t] = Mfma<T>::mma(av, breg[t][s], acc[t]);
#pragma unroll
            for (int j = 0; j < NREM; ++j) pr[j] += av * brem[j][s];
        }
#pragma unroll
        for (int t = 0; t < NATM; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * sl + Mfma<T>::RB * kq + Mfma<T>::RS * i, a = 16 * t + r16;
                if (x < NX && a < P) store(x, a, acc[t][i]);
            }
#pragma unroll
        for (int j = 0; j < NREM; ++j) {
            const T v = kq_sum(pr[j]);
            if (kq == 0 && xa < NX) store(xa, 16 * NATM + j, v);
        }
    }
}

// Plane-wave contraction over a full index m = -NF..NF with the conjugated
// exponentials B[m][a] = conj(E[m][a]), E[-m] = conj(E[m]):
//   sum_m B[m] X[m] = sum_{m >= 0} Br[m] s[m] + i Bi[m] d[m],
//   s[m] = X[m] + X[-m], d[m] = X[m] - X[-m] (s[0] = X[0], d[0] = 0),
// so that the complex product runs over NF + 1 values of m with the real
// matrices Br, Bi:  Re Y = Br.Re s - Bi.Im d,  Im Y = Br.Im s + Bi.Re d.
// Br, Bi point at the rows m = 0..NF (row stride P); X(x, k) takes the stored
// index k = m + NF.  Half the matrix-core work of the plain complex product.
// PF: the operands of the wave's next slab are loaded before the current
// slab's products (for X in global memory: hides the load latency).
template <int NWV, int P, int NX, int NF, bool PF, typename XR, typename XI, typename SF, typename T>
__device__ inline void mma_herm_store(XR Xr, XI Xi, const T *Br, const T *Bi, SF store, int nx = NX)
{
    constexpr int NATM = ColSplit<P>::NATM, NREM = ColSplit<P>::NREM, NRA = ColSplit<P>::NRA;
    constexpr int NH = NF + 1, NKS = (NH + 3) / 4;
    const int NSL = (nx + 15) / 16;  // slabs holding the nx live rows
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    T br[NATM][NKS], bi[NATM][NKS], rr[NRA][NKS], ri[NRA][NKS];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int k = 4 * s + kq;
#pragma unroll
        for (int t = 0; t < NATM; ++t) {
            const int a = 16 * t + r16;
            const bool ok = k < NH && a < P;
            br[t][s] = ok ? Br[k * P + a] : T(0);
            bi[t][s] = ok ? Bi[k * P + a] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NREM; ++j) {
            rr[j][s] = (k < NH) ? Br[k * P + 16 * NATM + j] : T(0);
            ri[j][s] = (k < NH) ? Bi[k * P + 16 * NATM + j] : T(0);
        }
    }
    // raw operands X[+m], X[-m] of a slab (X[-0] = 0: then s = d = X[0], and
    // the Bi row of m = 0 is zero, so d drops out there)
    auto fetch = [&](int sl, T (&fpr)[NKS], T (&fpi)[NKS], T (&fqr)[NKS], T (&fqi)[NKS]) {
        const int xa = 16 * sl + r16;
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int m = 4 * s + kq;
            const bool ok = sl < NSL && xa < nx && m < NH, okq = ok && m > 0;
            fpr[s] = ok ? Xr(xa, NF + m) : T(0);
            fpi[s] = ok ? Xi(xa, NF + m) : T(0);
            fqr[s] = okq ? Xr(xa, NF - m) : T(0);
            fqi[s] = okq ? Xi(xa, NF - m) : T(0);
        }
    };
    T pr[NKS], pi[NKS], qr[NKS], qi[NKS];
    if (PF) fetch(w, pr, pi, qr, qi);
    for (int sl = w; sl < NSL; sl += NWV) {
        const int xa = 16 * sl + r16;
        T npr[NKS], npi[NKS], nqr[NKS], nqi[NKS];
        if (PF) fetch(sl + NWV, npr, npi, nqr, nqi);
        else fetch(sl, pr, pi, qr, qi);
        v4_t<T> cr[NATM], ci[NATM];
        T ar[NRA], ai[NRA];
#pragma unroll
        for (int t = 0; t < NATM; ++t) cr[t] = ci[t] = v4_t<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < NRA; ++j) ar[j] = ai[j] = T(0);
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const T sr = pr[s] + qr[s], si = pi[s] + qi[s], dr = pr[s] - qr[s], ndi = qi[s] - pi[s];
#pragma unroll
            for (int t = 0; t < NATM; ++t) {
                cr[t] = Mfma<T>::mma(sr, br[t][s], cr[t]);
                cr[t] = Mfma<T>::mma(ndi, bi[t][s], cr[t]);
                ci[t] = Mfma<T>::mma(si, br[t][s], ci[t]);
                ci[t] = Mfma<T>::mma(dr, bi[t][s], ci[t]);
            }
#pragma unroll
            for (int j = 0; j < NREM; ++j) {
                ar[j] += sr * rr[j][s] + ndi * ri[j][s];
                ai[j] += si * rr[j][s] + dr * ri[j][s];
            }
        }
#pragma unroll
        for (int t = 0; t < NATM; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * sl + Mfma<T>::RB * kq + Mfma<T>::RS * i, a = 16 * t + r16;
                if (x < nx && a < P) store(x, a, cr[t][i], ci[t][i]);
            }
#pragma unroll
        for (int j = 0; j < NREM; ++j) {
            const T vr = kq_sum(ar[j]), vi = kq_sum(ai[j]);
            if (kq == 0 && xa < nx) store(xa, 16 * NATM + j, vr, vi);
        }
        if (PF) {
#pragma unroll
            for (int s = 0; s < NKS; ++s) { pr[s] = npr[s]; pi[s] = npi[s]; qr[s] = nqr[s]; qi[s] = nqi[s]; }
        }
    }
}

// COH: the anchor above the box was computed by the same launch (queue-fed)
template <typename T, int P, int NF, bool COH>
__device__ __forceinline__ void local_box_mfma(const Dev<T> &D, const int32_t B, const int level)
{
    using L = LocalMfma<T, P, NF>;
    constexpr int P2 = L::P2, P3 = L::P3, NN = L::NN, NH = L::NH, NM = L::NM, NSW = L::NSW;
    constexpr int NATM = ColSplit<P>::NATM, NREM = ColSplit<P>::NREM, NRA = ColSplit<P>::NRA;
    constexpr int G = L::G, KP = L::KP, NSL = L::NSL, NWV = L::NWV, NT = L::NT;
    extern __shared__ __align__(16) unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    T *Br1 = sm, *Bi1 = Br1 + NN * P;  // conj(E): B(k = m, a = j) = Er[m][j] - i Ei[m][j]
    T *B3 = Bi1 + NN * P;              // [KP][P]: c_m3 Er[m3][j3], then c_m3 Ei[m3][j3]
    T *Bx = B3 + KP * P, *By = Bx + P2, *Bz = By + P2;  // B(k = a, col = i) = M_d[i][a]
    T *xc = Bz + P2, *bw = xc + P;
    T *work = bw + P;
    // the parent anchor's values, loaded first so that their latency overlaps
    // the table set-up and the Lagrange rows
    constexpr int NVP = (P3 + NT - 1) / NT;
    T vpre[NVP];
    const int32_t A = level > 0 ? D.anchor[D.parent[B]] : -1;
    if (level > 0) {
        const T *src = D.local + (int64_t)D.local_slot[A] * P3;
#pragma unroll
        for (int i = 0; i < NVP; ++i) {
            const int t = threadIdx.x + i * NT;
            vpre[i] = t < P3 ? ld_c<COH>(src + t) : T(0);
        }
    }
    for (int t = threadIdx.x; t < NN * P; t += NT) {
        Br1[t] = D.epw[2 * t];
        Bi1[t] = -D.epw[2 * t + 1];
    }
    for (int t = threadIdx.x; t < KP * P; t += NT) {
        const int k = t / P, j = t % P, m3 = (k < NH) ? k : k - NH;
        const T cm = (m3 == 0) ? T(1) : T(2);
        const T *e = D.epw + 2 * ((m3 + NF) * P + j);
        B3[t] = cm * ((k < NH) ? e[0] : e[1]);
    }
    for (int t = threadIdx.x; t < P; t += NT) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    // the box's values: columns j3 < 16 NATM in MFMA fragments, the last
    // NREM columns in accr (row 16 sl + r16, the same in the row's four lanes)
    v4_t<T> acc[NSW][NATM];
    T accr[NSW][NRA];
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
#pragma unroll
        for (int t = 0; t < NATM; ++t) acc[i][t] = v4_t<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < NRA; ++j) accr[i][j] = T(0);
    }
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    __syncthreads();
    if (level == 0) {
        // root: the windowed W_0 values, in the fragment layout of the last step
        const T *w0B = D.w0vals + (int64_t)B * P3;  // root B = problem B
#pragma unroll
        for (int i = 0; i < NSW; ++i) {
            const int sl = w + NWV * i;
            if (sl >= NSL) break;
#pragma unroll
            for (int t = 0; t < NATM; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = 16 * sl + Mfma<T>::RB * kq + Mfma<T>::RS * q, a = 16 * t + r16;
                    if (x < P2 && a < P) acc[i][t][q] = w0B[x * P + a];
                }
            const int xa = 16 * sl + r16;
#pragma unroll
            for (int j = 0; j < NREM; ++j) accr[i][j] = (xa < P2) ? w0B[xa * P + 16 * NATM + j] : T(0);
        }
    } else {
        // interpolation from the anchor A of the parent: node i of B sits at
        // A-coordinate ((c_B + s_B x_i / 2) - c_A) * 2 / s_A
        const double sB = box_side(level), sA = box_side(D.blevel[A]);
        for (int t = threadIdx.x; t < 3 * P; t += NT) {
            const int d = t / P, i = t % P;
            const double xi = (D.bcenter[3 * (int64_t)B + d] + 0.5 * sB * D.xcheb64[i] - D.bcenter[3 * (int64_t)A + d]) *
                              (2.0 / sA);
            T row[P];
            lagrange_row<T>(P, xc, bw, (T)xi, row);
            T *Bd = (d == 0) ? Bx : (d == 1) ? By : Bz;
#pragma unroll
            for (int a = 0; a < P; ++a) Bd[a * P + i] = row[a];
        }
        T *vA = work, *t1 = work + P3;
#pragma unroll
        for (int i = 0; i < NVP; ++i) {
            const int t = threadIdx.x + i * NT;
            if (t < P3) vA[t] = vpre[i];
        }
        __syncthreads();
        // x: t1[i0][(a1 a2)] = sum_a0 vA[a0][(a1 a2)] Mx[i0][a0]
        mma_real_store<NWV, P, P2, P>([&](int x, int k) { return vA[k * P2 + x]; }, Bx,
                                      [&](int x, int a, T v) { t1[a * P2 + x] = v; });
        __syncthreads();
        // y: t2[i0][i1][a2] = sum_a1 t1[i0][a1][a2] My[i1][a1]; rows x = (i0, a2)
        T *t2 = vA;
        mma_real_store<NWV, P, P2, P>([&](int x, int k) { return t1[(x / P) * P2 + k * P + (x % P)]; }, By,
                                      [&](int x, int a, T v) { t2[(x / P) * P2 + a * P + (x % P)] = v; });
        __syncthreads();
        // z: acc[(i0 i1)][i2] = sum_a2 t2[(i0 i1)][a2] Mz[i2][a2]
        mma_real_acc<NWV, P, P2, P, NSW>([&](int x, int k) { return t2[x * P + k]; }, Bz, acc, accr);
    }
    if (D.psi_slot[B] >= 0) {
        const int64_t nm = D.pwstride;
        const T *psr = D.psi + 2 * (int64_t)D.psi_slot[B] * nm, *psi = psr + nm;
        T *A1r = work, *A1i = work + P * NM, *B2 = work + 2 * P * NM;
        __syncthreads();
        // m1: A1[j1][(m3 m2)] = sum_m1 conj(E[m1][j1]) Psi[m1][(m3 m2)], Psi read from HBM
        mma_herm_store<NWV, P, NM, NF, true>([&](int x, int k) { return psr[k * NM + x]; },
                                            [&](int x, int k) { return psi[k * NM + x]; }, Br1 + NF * P, Bi1 + NF * P,
                                                   [&](int x, int a, T vr, T vi) {
            A1r[a * NM + x] = vr;
            A1i[a * NM + x] = vi;
        });
        // m2 then m3, G values of j1 at a time (G p rows: whole slabs)
        for (int g0 = 0; g0 < P; g0 += G) {
            const int g = min(G, P - g0);
            __syncthreads();
            // m2: B2[(j1 j2)][m3 | NH + m3] = sum_m2 conj(E[m2][j2]) A1[j1][m3][m2]; rows x = (j1 - g0, m3)
            mma_herm_store<NWV, P, G * NH, NF, false>(
                [&](int x, int k) { return (x < g * NH) ? A1r[(g0 * NH + x) * NN + k] : T(0); },
                [&](int x, int k) { return (x < g * NH) ? A1i[(g0 * NH + x) * NN + k] : T(0); }, Br1 + NF * P,
                Bi1 + NF * P,
                [&](int x, int a, T vr, T vi) {
                    if (x < g * NH) {
                        const int j1 = x / NH, m3 = x % NH;
                        B2[(j1 * P + a) * KP + m3] = vr;
                        B2[(j1 * P + a) * KP + NH + m3] = vi;
                    }
                },
                g * NH);
            __syncthreads();
            // m3: acc[(j1 j2)][j3] += sum_k' B2[(j1 j2)][k'] B3[k'][j3] for the slabs of this group
            constexpr int NKS = (KP + 3) / 4;
            T breg[NATM][NKS], brem[NRA][NKS];
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                const int k = 4 * s + kq;
#pragma unroll
                for (int t = 0; t < NATM; ++t) {
                    const int a = 16 * t + r16;
                    breg[t][s] = (k < KP && a < P) ? B3[k * P + a] : T(0);
                }
#pragma unroll
                for (int j = 0; j < NREM; ++j) brem[j][s] = (k < KP) ? B3[k * P + 16 * NATM + j] : T(0);
            }
            const int r0 = g0 * P, r1 = (g0 + g) * P;  // rows of this group, multiples of 16 at r0
#pragma unroll
            for (int i = 0; i < NSW; ++i) {
                const int sl = w + NWV * i;
                if (sl >= NSL || 16 * sl < r0 || 16 * sl >= r1) continue;  // uniform in the wave
                const int xa = 16 * sl + r16;
                T pr[NRA];
#pragma unroll
                for (int j = 0; j < NRA; ++j) pr[j] = T(0);
#pragma unroll
                for (int s = 0; s < NKS; ++s) {
                    const int k = 4 * s + kq;
                    const T av = (xa < r1 && k < KP) ? B2[(xa - r0) * KP + k] : T(0);
#pragma unroll
                    for (int t = 0; t < NATM; ++t)
                        acc[i][t] = Mfma<T>::mma(av, breg[t][s], acc[i][t]);
#pragma unroll
                    for (int j = 0; j < NREM; ++j) pr[j] += av * brem[j][s];
                }
#pragma unroll
                for (int j = 0; j < NREM; ++j) accr[i][j] += kq_sum(pr[j]);
            }
        }
    }
    // the box's values, x-major p^3 block: straight from the fragments, or
    // (COH, and a finer anchor of the same launch reads them) through LDS
    // and out in whole lines with cache-bypassing stores; atomic stores
    // straight from the fragments keep their order and cost this kernel
    // registers
    T *dst = D.local + (int64_t)D.local_slot[B] * P3;
    const bool coh = COH && D.anc_read[D.local_slot[B]];
    T *out = dst;
    if (coh) {
        out = work;
        __syncthreads();  // the last group's B2 reads are done
    }
#pragma unroll
    for (int i = 0; i < NSW; ++i) {
        const int sl = w + NWV * i;
        if (sl >= NSL) break;
#pragma unroll
        for (int t = 0; t < NATM; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x = 16 * sl + Mfma<T>::RB * kq + Mfma<T>::RS * q, a = 16 * t + r16;
                if (x < P2 && a < P) out[x * P + a] = acc[i][t][q];
            }
        const int xa = 16 * sl + r16;
#pragma unroll
        for (int j = 0; j < NREM; ++j)
            if (kq == 0 && xa < P2) out[xa * P + 16 * NATM + j] = accr[i][j];
    }
    if (coh) {
        __syncthreads();
        for (int t = threadIdx.x; t < P3; t += NT) st_c<true>(dst + t, work[t]);
    }
}

// FP32: 4 waves per SIMD (two blocks per CU); FP64: two (LDS and registers
// take one block per CU)
template <typename T>
constexpr int local_waves() { return sizeof(T) == 4 ? 4 : 2; }

template <typename T, int P, int NF>
__global__ void __launch_bounds__(LOCAL_NT, local_waves<T>()) k_local_mfma(Dev<T> D, const int32_t *list, int level)
{
    local_box_mfma<T, P, NF, false>(D, list[blockIdx.x], level);
}

// one box per workgroup (grid = anchors), taken from the queue: looping over
// boxes in one workgroup held the body's loop-invariant index arithmetic in
// registers across items and pushed this kernel into scratch
template <typename T, int P, int NF>
__global__ void __launch_bounds__(LOCAL_NT, local_waves<T>()) k_local_mfma_q(Dev<T> D, WorkQ q)
{
    queue_item(
        q,
        [&](int32_t B) {
            if (threadIdx.x == 0 && D.blevel[B] > 0) wait_done(q, D.anchor[D.parent[B]]);
        },
        [&](int32_t B) { local_box_mfma<T, P, NF, true>(D, B, D.blevel[B]); });
}

// ------------------------------------ outgoing plane waves on matrix cores
// Proxy -> plane waves (eq. outgoingexpansion2) on MFMA, three mode
// products in the fragment scheme of the local stage:
//   j3 -> m3  A[(j1 j2)][m3 | NH + m3] = sum_j3 rho[(j1 j2)][j3] (Re | Im) E[m3][j3]
//   j2 -> m2  B2[(mm j1)][m2] = sum_j2 A[(j1 j2)][m3] E[m2][j2]   (complex)
//   j1 -> m1  Phi[m1][(mm m2)] = sum_j1 E[m1][j1] B2[(mm j1)][m2] (complex)
// the last two for G values of m3 at a time; each group's Phi rows are
// staged in LDS and written to HBM as contiguous runs of G * nn values.
// Forward plane-wave contraction to a full output index m = -NF..NF:
// Y[m] = sum_k E[m][k] X[k] with E[-m] = conj(E[m]) needs only the real
// matrices Er, Ei at m >= 0:  U = Er.X, V = Ei.X (X complex),
//   Y[m] = U + i V,  Y[-m] = U - i V,
// which halves the matrix-core work of the plain complex product.  Br, Bi
// point at column m = 0 of E (element (k, m) at k * NBS + m); store receives
// (x, m, Y[m], Y[-m]) for m = 0..NF (Y[-0] is Y[0]).
template <int NWV, int NF, int NX, int NK, int NBS, typename XR, typename XI, typename SF, typename T>
__device__ inline void mma_herm_out_store(XR Xr, XI Xi, const T *Br, const T *Bi, SF store, int nx = NX)
{
    constexpr int NH = NF + 1, NKS = (NK + 3) / 4, NAT = (NH + 15) / 16;
    const int NSL = (nx + 15) / 16;  // slabs holding the nx live rows
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    T br[NAT][NKS], bi[NAT][NKS];
#pragma unroll
    for (int t = 0; t < NAT; ++t)
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kq, a = 16 * t + r16;
            const bool ok = k < NK && a < NH;
            br[t][s] = ok ? Br[k * NBS + a] : T(0);
            bi[t][s] = ok ? Bi[k * NBS + a] : T(0);
        }
    for (int sl = w; sl < NSL; sl += NWV) {
        const int xa = 16 * sl + r16;
        v4_t<T> ur[NAT], ui[NAT], vr[NAT], vi[NAT];
#pragma unroll
        for (int t = 0; t < NAT; ++t) ur[t] = ui[t] = vr[t] = vi[t] = v4_t<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kq;
            const bool ok = xa < nx && k < NK;
            const T ar = ok ? Xr(xa, k) : T(0), ai = ok ? Xi(xa, k) : T(0);
#pragma unroll
            for (int t = 0; t < NAT; ++t) {
                ur[t] = Mfma<T>::mma(ar, br[t][s], ur[t]);
                ui[t] = Mfma<T>::mma(ai, br[t][s], ui[t]);
                vr[t] = Mfma<T>::mma(ar, bi[t][s], vr[t]);
                vi[t] = Mfma<T>::mma(ai, bi[t][s], vi[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < NAT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * sl + Mfma<T>::RB * kq + Mfma<T>::RS * i, m = 16 * t + r16;
                if (x < nx && m < NH)
                    store(x, m, ur[t][i] - vi[t][i], ui[t][i] + vr[t][i], ur[t][i] + vi[t][i], ui[t][i] - vr[t][i]);
            }
    }
}

constexpr int P2PW_NT = 512;  // threads per block of proxy -> plane waves on matrix cores

template <typename T, int P, int NF>
struct P2pwMfma {
    static constexpr int P2 = P * P, P3 = P2 * P, NN = 2 * NF + 1, NH = NF + 1, NM = NH * NN, W1 = 2 * NH;
    static constexpr int G = 4;
    static constexpr int R0 = (P3 > 2 * P * G * NN + 2 * NN * G * NN) ? P3 : 2 * P * G * NN + 2 * NN * G * NN;
    static constexpr int TAB = P * W1 + 2 * P * NN;
    static size_t lds() { return sizeof(T) * (TAB + R0 + P2 * W1); }
};

template <typename T, int P, int NF>
__global__ void __launch_bounds__(P2PW_NT) k_proxy2pw_mfma(Dev<T> D, const int32_t *list)
{
    using L = P2pwMfma<T, P, NF>;
    constexpr int P2 = L::P2, P3 = L::P3, NN = L::NN, NH = L::NH, NM = L::NM, W1 = L::W1, G = L::G;
    extern __shared__ __align__(16) unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    T *B1 = sm;                    // [j3][W1]: Re E[m3][j3] | Im E[m3][j3]
    T *BrT = B1 + P * W1;          // [j][m]: Re E[m][j]
    T *BiT = BrT + P * NN;         //         Im E[m][j]
    T *r0 = BiT + P * NN;          // rho, then B2 and the staged Phi rows
    T *A = r0 + L::R0;             // [(j1 j2)][W1]
    T *B2r = r0, *B2i = B2r + P * G * NN;       // [(mm j1)][m2]
    T *Fr = B2i + P * G * NN, *Fi = Fr + NN * G * NN;  // [m1][(mm m2)]
    const int32_t B = list[blockIdx.x];
    for (int t = threadIdx.x; t < P * W1; t += P2PW_NT) {
        const int j = t / W1, a = t % W1, m3 = (a < NH) ? a : a - NH;
        B1[t] = D.epw[2 * ((m3 + NF) * P + j) + (a < NH ? 0 : 1)];
    }
    for (int t = threadIdx.x; t < P * NN; t += P2PW_NT) {
        const int j = t / NN, m = t % NN;
        BrT[t] = D.epw[2 * (m * P + j)];
        BiT[t] = D.epw[2 * (m * P + j) + 1];
    }
    const T *src = D.proxy + (int64_t)D.proxy_slot[B] * P3;
    for (int t = threadIdx.x; t < P3; t += P2PW_NT) r0[t] = src[t];
    __syncthreads();
    // j3 -> m3 (real rho times the real and imaginary rows)
    mma_real_store<P2PW_NT / 64, W1, P2, P>([&](int x, int k) { return r0[x * P + k]; }, B1,
                                              [&](int x, int a, T v) { A[x * W1 + a] = v; });
    const int64_t nm = D.pwstride;
    T *outr = D.phi + 2 * (int64_t)D.proxy_slot[B] * nm;
    T *outi = outr + nm;
    for (int g0 = 0; g0 < NH; g0 += G) {
        const int g = min(G, NH - g0);
        __syncthreads();
        // j2 -> m2: rows x = (mm, j1), the g P live rows first
        mma_herm_out_store<P2PW_NT / 64, NF, P * G, P, NN>(
            [&](int x, int k) { const int mm = x / P, j1 = x % P; return (mm < g) ? A[(j1 * P + k) * W1 + g0 + mm] : T(0); },
            [&](int x, int k) { const int mm = x / P, j1 = x % P; return (mm < g) ? A[(j1 * P + k) * W1 + NH + g0 + mm] : T(0); },
            BrT + NF, BiT + NF, [&](int x, int m, T pr, T pi, T nr, T ni) {
                B2r[x * NN + NF + m] = pr;
                B2i[x * NN + NF + m] = pi;
                if (m > 0) {
                    B2r[x * NN + NF - m] = nr;
                    B2i[x * NN + NF - m] = ni;
                }
            },
            P * g);
        __syncthreads();
        // j1 -> m1: rows x = (mm, m2)
        mma_herm_out_store<P2PW_NT / 64, NF, G * NN, P, NN>(
            [&](int x, int k) { const int mm = x / NN, m2 = x % NN; return (mm < g) ? B2r[(mm * P + k) * NN + m2] : T(0); },
            [&](int x, int k) { const int mm = x / NN, m2 = x % NN; return (mm < g) ? B2i[(mm * P + k) * NN + m2] : T(0); },
            BrT + NF, BiT + NF, [&](int x, int m, T pr, T pi, T nr, T ni) {
                Fr[(NF + m) * G * NN + x] = pr;
                Fi[(NF + m) * G * NN + x] = pi;
                if (m > 0) {
                    Fr[(NF - m) * G * NN + x] = nr;
                    Fi[(NF - m) * G * NN + x] = ni;
                }
            },
            g * NN);
        __syncthreads();
        // the group's rows of Phi[m1][m3][m2]: runs of g * nn values per m1
        for (int t = threadIdx.x; t < NN * g * NN; t += P2PW_NT) {
            const int m1 = t / (g * NN), r = t % (g * NN);
            outr[(int64_t)m1 * NM + g0 * NN + r] = Fr[m1 * G * NN + r];
            outi[(int64_t)m1 * NM + g0 * NN + r] = Fi[m1 * G * NN + r];
        }
    }
}

// ------------------------------------------------------------ leaf targets


// -------------------------------------------------------------- residual
// One workgroup per target leaf.  The sources of the leaf's gather list are
// staged in LDS, a round of TPB list entries at a time, keeping only those
// that can reach the leaf: the residual vanishes beyond the source box side
// s, so a source farther than s from the bounding box of the leaf's targets
// contributes nothing (on clustered points this drops about 37 % of the
// candidate pairs).  Staged points are offsets from the leaf centre formed in
// FP64 and rounded to T once per point, with 1/s of the source box level, a
// power of two, so t = r^2 (1/s)^2 is formed exactly in the loop; each
// thread then sums one target against a stride of the staged sources, and
// the per-pass partial sums are added into an FP64 accumulator.  Five staged
// arrays of 512 values (the partial-sum buffer reuses them) and the list
// offsets keep the LDS of an FP32 block near 10 KB, so that many blocks share
// a compute unit, also beside the far-field kernels.

// 1/sqrt in the working precision (the float overload is the hardware
// reciprocal square root, about 1 ulp, without the rescaling for denormal
// arguments: r^2 > 0 here is a squared distance between distinct points)
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return rsqrt(x); }

// g(t) = Phi(sqrt t)/sqrt t is evaluated by Horner's rule in u = 2t - 1 from
// its power-series coefficients in u (converted on the host from the
// Chebyshev series).  The function is well conditioned in that basis: the
// sum of |a_k| stays within 0.2 % of max |g| for tolerances 1e-3 .. 1e-12,
// so Horner is as accurate as Clenshaw's recurrence at half its operations.
// DEG: compile-time degree bucket (coefficients above the plan's degree are
// zero, which leaves the result unchanged); the coefficients live in registers.
template <typename T, int DEG, int POW>
__global__ void __launch_bounds__(TPB) k_residual(Dev<T> D, const int32_t *leaves, const int32_t *nl_off,
                                                  const int32_t *nl_src, const int32_t *nl_pre)
{
    // sources staged per pass (10 KB of LDS in FP32: more blocks share a
    // compute unit; 1024 was 6 % slower, 256 slower too)
    constexpr int RCAP = 512;
    // staged sources (sis: 1/s of the source box); the per-split partial
    // sums reuse their space once a target chunk is done
    __shared__ union {
        struct { T x[RCAP], y[RCAP], z[RCAP], q[RCAP], is[RCAP]; } s;
        double part[TPB];
    } stg;
    T *sx = stg.s.x, *sy = stg.s.y, *sz = stg.s.z, *sq = stg.s.q, *sis = stg.s.is;
    double *part = stg.part;
    // running source counts of the block's list (L + 1 entries), then the
    // entries' first points and levels (L each): dynamic LDS, sized at
    // launch to the plan's longest list
    extern __shared__ __align__(16) int32_t loff[];
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = D.tstart[B];  // the leaf's targets
    const int nt = D.tcount[B];
    const int32_t l0 = nl_off[blockIdx.x];
    const int L = nl_off[blockIdx.x + 1] - l0;
    T gc[DEG + 1];
#pragma unroll
    for (int k = 0; k <= DEG; ++k) gc[k] = (k <= D.gdeg) ? D.gmono[k] : T(0);
    // running source counts over the list (computed at plan time), and each
    // entry's first point and level, so that staging a source takes one
    // dependent global load (its coordinates) instead of three
    int32_t *lbeg = loff + L + 1, *llev = lbeg + L;
    for (int k = threadIdx.x; k <= L; k += TPB) loff[k] = nl_pre[l0 + blockIdx.x + k];
    for (int k = threadIdx.x; k < L; k += TPB) {
        const int32_t Tb = nl_src[l0 + k];
        lbeg[k] = D.pstart[Tb];
        llev[k] = D.blevel[Tb];
    }
    __syncthreads();
    const int nsrc = loff[L];
    const double cx = D.bcenter[3 * (int64_t)B], cy = D.bcenter[3 * (int64_t)B + 1], cz = D.bcenter[3 * (int64_t)B + 2];
    // one thread per target and source share; a leaf of nt <= 64 targets uses
    // TPB/nt shares so that few threads idle
    const int tch = min(max(nt, 1), 64);
    const int nsplit = TPB / tch;
    const int tl = threadIdx.x % tch, split = threadIdx.x / tch;
    __shared__ int wtot[TPB / 64];
    __shared__ T tbb[6];  // the target chunk's bounding box: low corner, high corner
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int tbase = 0; tbase < nt; tbase += tch) {
        const bool active = (tbase + tl) < nt;
        const int64_t it = t0 + tbase + (active ? tl : 0);
        const T xt = (T)(D.Xt[it] - cx), yt = (T)(D.Yt[it] - cy), zt = (T)(D.Zt[it] - cz);
        // bounding box of the chunk's targets (wave 0 holds them all: tch <= 64)
        if (wv == 0) {
            T b[6] = {xt, yt, zt, -xt, -yt, -zt};
#pragma unroll
            for (int d = 1; d < 64; d <<= 1)
#pragma unroll
                for (int k = 0; k < 6; ++k) b[k] = min(b[k], __shfl_xor(b[k], d));
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    tbb[k] = b[k];
                    tbb[3 + k] = -b[3 + k];
                }
            }
        }
        double acc = 0.0;
        for (int cursor = 0; cursor < nsrc;) {
            // stage the next sources of the list that can reach the box: a
            // source farther than its range s from the box is farther than s
            // from every target (the distance to the box is formed with the
            // same rounded operations as the pair distance, so it is not
            // larger than any pair's; the margin keeps the comparison safe)
            int cnt = 0;
            __syncthreads();
            while (cursor < nsrc && cnt <= RCAP - TPB) {
                const int g = cursor + threadIdx.x;
                bool keep = false;
                T ux = T(0), uy = T(0), uz = T(0), uq = T(0), uis = T(0);
                if (g < nsrc) {
                    int lo = 0, hi = L - 1;  // entry k with loff[k] <= g < loff[k+1]
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (loff[mid] <= g) lo = mid; else hi = mid - 1;
                    }
                    const int64_t j = (int64_t)lbeg[lo] + (g - loff[lo]);
                    ux = (T)(D.X[j] - cx);
                    uy = (T)(D.Y[j] - cy);
                    uz = (T)(D.Z[j] - cz);
                    uq = (T)D.qs[j];
                    uis = (T)ldexp(1.0, llev[lo]);
                    const T ex = max(max(tbb[0] - ux, T(0)), ux - tbb[3]);
                    const T ey = max(max(tbb[1] - uy, T(0)), uy - tbb[4]);
                    const T ez = max(max(tbb[2] - uz, T(0)), uz - tbb[5]);
                    const T d2 = ex * ex + ey * ey + ez * ez;
                    keep = d2 * uis * uis < T(1.0001);
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
                    sz[pos] = uz;
                    sq[pos] = uq;
                    sis[pos] = uis;
                }
                cnt += total;
                cursor += TPB;
                __syncthreads();
            }
            T pacc = T(0);
            // RB candidates per round: their operands are read and tested
            // together (independent LDS reads in flight), then the pairs in
            // range are summed one by one
            constexpr int RB = 4;
            for (int j0 = split; j0 < cnt && split < nsplit; j0 += RB * nsplit) {
                T r2v[RB], ttv[RB];
                int jv[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int j = j0 + u * nsplit;
                    jv[u] = j < cnt ? j : -1;
                    const int jj = j < cnt ? j : j0;  // a valid slot for the spare lanes
                    const T dx = xt - sx[jj], dy = yt - sy[jj], dz = zt - sz[jj];
                    r2v[u] = dx * dx + dy * dy + dz * dz;
                    const T is = sis[jj];
                    ttv[u] = r2v[u] * is * is;
                }
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    if (jv[u] >= 0 && ttv[u] < T(1)) {
                        const int j = jv[u];
                        // Horner for g(t) = Phi(sqrt t)/sqrt t in u = 2t - 1
                        const T uu = T(2) * ttv[u] - T(1);
                        T g = gc[DEG];
#pragma unroll
                        for (int k = DEG - 1; k >= 0; --k) g = g * uu + gc[k];
                        if constexpr (POW == 1) {  // 1/r - g(t)/s
                            const T rinv = (r2v[u] > T(0)) ? rsq(r2v[u]) : T(0);
                            pacc += sq[j] * (rinv - g * sis[j]);
                        } else {  // 1/r^2 - g2(t)/s^2
                            const T r2inv = (r2v[u] > T(0)) ? T(1) / r2v[u] : T(0);
                            pacc += sq[j] * (r2inv - g * sis[j] * sis[j]);
                        }
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

// Residual sums of the Yukawa kernel: e^{-lambda r}/r - M_l(r) for
// 0 < r < s_l and -M_l(0) at r = 0, M_l(x s_l) = m_l(x)/s_l from the level's
// Chebyshev series in u = 2x^2 - 1 (all levels' series in LDS).  Gather lists,
// staging and thread layout as in k_residual.
template <typename T>
__global__ void __launch_bounds__(TPB) k_residual_y3(Dev<T> D, const int32_t *leaves, const int32_t *nl_off,
                                                     const int32_t *nl_src, const int32_t *nl_pre)
{
    constexpr int RCAP = 512, YLEV = 32, YC = 48;
    __shared__ union {
        struct { T x[RCAP], y[RCAP], z[RCAP], q[RCAP], is[RCAP]; } s;
        double part[TPB];
    } stg;
    __shared__ T yc[YLEV * YC];
    __shared__ T yself[YLEV];
    __shared__ int8_t slev[RCAP];
    T *sx = stg.s.x, *sy = stg.s.y, *sz = stg.s.z, *sq = stg.s.q, *sis = stg.s.is;
    double *part = stg.part;
    extern __shared__ __align__(16) int32_t loff[];
    __shared__ int wtot[TPB / 64];
    __shared__ T tbb[6];  // the target chunk's bounding box: low corner, high corner
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = D.tstart[B];  // the leaf's targets
    const int nt = D.tcount[B];
    const int32_t l0 = nl_off[blockIdx.x];
    const int L = nl_off[blockIdx.x + 1] - l0;
    const int deg = D.ydeg;
    for (int k = threadIdx.x; k < D.ynlev * YC; k += TPB) yc[k] = D.ycheb[k];
    for (int k = threadIdx.x; k < D.ynlev; k += TPB) yself[k] = (T)D.yself[k];
    // the entries' first points and levels after the running counts (one
    // dependent global load per staged source)
    int32_t *lbeg = loff + L + 1, *llev = lbeg + L;
    for (int k = threadIdx.x; k <= L; k += TPB) loff[k] = nl_pre[l0 + blockIdx.x + k];
    for (int k = threadIdx.x; k < L; k += TPB) {
        const int32_t Tb = nl_src[l0 + k];
        lbeg[k] = D.pstart[Tb];
        llev[k] = D.blevel[Tb];
    }
    __syncthreads();
    const int nsrc = loff[L];
    const T lam = (T)D.ylam;
    const double cx = D.bcenter[3 * (int64_t)B], cy = D.bcenter[3 * (int64_t)B + 1], cz = D.bcenter[3 * (int64_t)B + 2];
    const int tch = min(max(nt, 1), 64);
    const int nsplit = TPB / tch;
    const int tl = threadIdx.x % tch, split = threadIdx.x / tch;
    for (int tbase = 0; tbase < nt; tbase += tch) {
        const bool active = (tbase + tl) < nt;
        const int64_t it = t0 + tbase + (active ? tl : 0);
        const T xt = (T)(D.Xt[it] - cx), yt = (T)(D.Yt[it] - cy), zt = (T)(D.Zt[it] - cz);
        // the chunk's bounding box (wave 0 holds all its targets: tch <= 64)
        if (wv == 0) {
            T b[6] = {xt, yt, zt, -xt, -yt, -zt};
#pragma unroll
            for (int d = 1; d < 64; d <<= 1)
#pragma unroll
                for (int q = 0; q < 6; ++q) b[q] = min(b[q], __shfl_xor(b[q], d));
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    tbb[q] = b[q];
                    tbb[3 + q] = -b[3 + q];
                }
            }
        }
        double acc = 0.0;
        for (int cursor = 0; cursor < nsrc;) {
            // stage the sources that can reach the box, as in k_residual
            int cnt = 0;
            __syncthreads();
            while (cursor < nsrc && cnt <= RCAP - TPB) {
                const int g = cursor + threadIdx.x;
                bool keep = false;
                T ux = T(0), uy = T(0), uz = T(0), uq = T(0), uis = T(0);
                int ulev = 0;
                if (g < nsrc) {
                    int lo = 0, hi = L - 1;  // entry k with loff[k] <= g < loff[k+1]
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (loff[mid] <= g) lo = mid; else hi = mid - 1;
                    }
                    const int64_t j = (int64_t)lbeg[lo] + (g - loff[lo]);
                    ulev = llev[lo];
                    ux = (T)(D.X[j] - cx);
                    uy = (T)(D.Y[j] - cy);
                    uz = (T)(D.Z[j] - cz);
                    uq = (T)D.qs[j];
                    uis = (T)ldexp(1.0, ulev);
                    const T ex = max(max(tbb[0] - ux, T(0)), ux - tbb[3]);
                    const T ey = max(max(tbb[1] - uy, T(0)), uy - tbb[4]);
                    const T ez = max(max(tbb[2] - uz, T(0)), uz - tbb[5]);
                    const T d2 = ex * ex + ey * ey + ez * ez;
                    keep = d2 * uis * uis < T(1.0001);
                }
                const uint64_t m = __ballot(keep);
                if (lane == 0) wtot[wv] = __popcll(m);
                __syncthreads();
                int before = 0, total = 0;
#pragma unroll
                for (int q = 0; q < TPB / 64; ++q) {
                    const int c = wtot[q];
                    before += q < wv ? c : 0;
                    total += c;
                }
                if (keep) {
                    const int pos = cnt + before + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                    sx[pos] = ux;
                    sy[pos] = uy;
                    sz[pos] = uz;
                    sq[pos] = uq;
                    sis[pos] = uis;
                    slev[pos] = (int8_t)ulev;
                }
                cnt += total;
                cursor += TPB;
                __syncthreads();
            }
            T pacc = T(0);
            for (int j = split; j < cnt && split < nsplit; j += nsplit) {
                const T dx = xt - sx[j], dy = yt - sy[j], dz = zt - sz[j];
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T is = sis[j];
                const T tt = r2 * is * is;
                if (tt < T(1)) {
                    const T *cf = yc + (int)slev[j] * YC;
                    T val;
                    if (r2 > T(0)) {
                        const T u = T(2) * tt - T(1);
                        T b1 = T(0), b2 = T(0);
                        for (int k = deg; k >= 1; --k) {
                            const T b0 = cf[k] + T(2) * u * b1 - b2;
                            b2 = b1;
                            b1 = b0;
                        }
                        const T r = sqrt(r2);
                        val = exp(-lam * r) / r - (cf[0] + u * b1 - b2) * is;
                    } else {
                        val = -yself[slev[j]];
                    }
                    pacc += sq[j] * val;
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

// ----------------------------------------------------------- root window
// Root proxies -> W_0 plane waves (spacing hw, half width nw) times the
// window weights -> values on the root grid, in FP64 (O(1) work per eval).
// Eight grid-wide stages, one thread per output entry; the intermediates
// live in a global scratch buffer laid out as in root_scratch_elems.
struct RootLayout {
    int64_t rows, rho, Ar, Ai, Br, Bi, Fr, Fi, C1r, C1i, C2r, C2i, total;
    __host__ __device__ RootLayout(int p, int n, int nh, int npts)
    {
        const int64_t p2 = (int64_t)p * p;
        rows = 0;
        rho = rows + 3 * (int64_t)npts * p;
        Ar = rho + p2 * p;
        Ai = Ar + p2 * nh;
        Br = Ai + p2 * nh;
        Bi = Br + (int64_t)p * nh * n;
        Fr = Bi + (int64_t)p * nh * n;
        Fi = Fr + (int64_t)n * nh * n;
        C1r = Fi + (int64_t)n * nh * n;
        C1i = C1r + (int64_t)n * n * p;
        C2r = C1i + (int64_t)n * n * p;
        C2i = C2r + (int64_t)n * p2;
        total = C2i + (int64_t)n * p2;
    }
};

template <typename T>
__global__ void __launch_bounds__(TPB) k_root_stage(Dev<T> D, int stage)
{
    // problem b = blockIdx.y: its root is box b, its scratch its own slice
    const int b = blockIdx.y;
    const int p = D.p, p2 = p * p, p3 = p2 * p, n = D.nwn, nh = D.nwh, nw = D.nw;
    const int npm = D.root_npmax;
    const RootLayout R(p, n, nh, npm);
    double *S = D.rootscratch + (int64_t)b * D.root_stride;
    const double *E = D.ew64;  // [n][p][2], rows m + nw
    const int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x;
    const bool root_fout = (D.bflags[b] & 2) != 0;
    const int npts = root_fout ? 0 : D.pcount[b];  // a root without F_out is a leaf of <= npm points
    const int64_t p0 = D.pstart[b];
    switch (stage) {
    case 0:  // Lagrange rows of the root's points (root without F_out)
        if (e < 3 * npts) {
            const int pt = (int)(e / 3), d = (int)(e % 3);
            const double x = (d == 0) ? D.X[p0 + pt] : (d == 1) ? D.Y[p0 + pt] : D.Z[p0 + pt];
            lagrange_row<double>(p, D.xcheb64, D.bary64, 2.0 * x, S + R.rows + (d * (int64_t)npm + pt) * p);
        }
        break;
    case 1:  // root proxies
        if (e < p3) {
            double v = 0.0;
            if (root_fout) {
                v = (double)D.proxy[(int64_t)D.proxy_slot[b] * p3 + e];
            } else {
                const int a0 = (int)(e / p2), a1 = (int)((e / p) % p), a2 = (int)(e % p);
                const double *Lx = S + R.rows, *Ly = Lx + (int64_t)npm * p, *Lz = Ly + (int64_t)npm * p;
                for (int pt = 0; pt < npts; ++pt)
                    v += Lx[pt * p + a0] * Ly[pt * p + a1] * Lz[pt * p + a2] * D.qs[p0 + pt];
            }
            S[R.rho + e] = v;
        }
        break;
    case 2:  // A[(j1 j2)][m3] = sum_j3 E[m3][j3] rho
        if (e < (int64_t)p2 * nh) {
            const int r = (int)(e / nh), m3 = (int)(e % nh);
            double re = 0, im = 0;
            for (int j = 0; j < p; ++j) {
                re += E[2 * ((m3 + nw) * p + j)] * S[R.rho + r * p + j];
                im += E[2 * ((m3 + nw) * p + j) + 1] * S[R.rho + r * p + j];
            }
            S[R.Ar + e] = re;
            S[R.Ai + e] = im;
        }
        break;
    case 3:  // B[j1][m3][m2] = sum_j2 E[m2][j2] A[j1][j2][m3]
        if (e < (int64_t)p * nh * n) {
            const int j1 = (int)(e / (nh * n)), m3 = (int)((e / n) % nh), m2 = (int)(e % n);
            double re = 0, im = 0;
            for (int j = 0; j < p; ++j) {
                const double er = E[2 * (m2 * p + j)], ei = E[2 * (m2 * p + j) + 1];
                const double ar = S[R.Ar + (j1 * p + j) * nh + m3], ai = S[R.Ai + (j1 * p + j) * nh + m3];
                re += er * ar - ei * ai;
                im += er * ai + ei * ar;
            }
            S[R.Br + e] = re;
            S[R.Bi + e] = im;
        }
        break;
    case 4:  // Phi[m1][m3][m2] = w(m) sum_j1 E[m1][j1] B[j1][m3][m2]
        if (e < (int64_t)n * nh * n) {
            const int m1 = (int)(e / (nh * n)), r = (int)(e % (nh * n)), m3 = r / n, m2 = r % n;
            double re = 0, im = 0;
            for (int j = 0; j < p; ++j) {
                const double er = E[2 * (m1 * p + j)], ei = E[2 * (m1 * p + j) + 1];
                const double br = S[R.Br + j * nh * n + r], bi = S[R.Bi + j * nh * n + r];
                re += er * br - ei * bi;
                im += er * bi + ei * br;
            }
            const double w = D.ww64[(m3 * n + m2) * n + m1];
            S[R.Fr + e] = re * w;
            S[R.Fi + e] = im * w;
        }
        break;
    case 5:  // C1[m1][m2][j3] = sum_m3 c_m3 conj(E[m3][j3]) Phi[m1][m3][m2]
        if (e < (int64_t)n * n * p) {
            const int m1 = (int)(e / (n * p)), m2 = (int)((e / p) % n), j3 = (int)(e % p);
            double re = 0, im = 0;
            for (int m3 = 0; m3 < nh; ++m3) {
                const double c = (m3 == 0) ? 1.0 : 2.0;
                const double er = c * E[2 * ((m3 + nw) * p + j3)], ei = -c * E[2 * ((m3 + nw) * p + j3) + 1];
                const double fr = S[R.Fr + (m1 * nh + m3) * n + m2], fi = S[R.Fi + (m1 * nh + m3) * n + m2];
                re += er * fr - ei * fi;
                im += er * fi + ei * fr;
            }
            S[R.C1r + e] = re;
            S[R.C1i + e] = im;
        }
        break;
    case 6:  // C2[m1][j2][j3] = sum_m2 conj(E[m2][j2]) C1[m1][m2][j3]
        if (e < (int64_t)n * p2) {
            const int m1 = (int)(e / p2), j2 = (int)((e / p) % p), j3 = (int)(e % p);
            double re = 0, im = 0;
            for (int m2 = 0; m2 < n; ++m2) {
                const double er = E[2 * (m2 * p + j2)], ei = -E[2 * (m2 * p + j2) + 1];
                const double cr = S[R.C1r + (m1 * n + m2) * p + j3], ci = S[R.C1i + (m1 * n + m2) * p + j3];
                re += er * cr - ei * ci;
                im += er * ci + ei * cr;
            }
            S[R.C2r + e] = re;
            S[R.C2i + e] = im;
        }
        break;
    case 7:  // values: Re sum_m1 conj(E[m1][j1]) C2[m1][(j2 j3)]
        if (e < p3) {
            const int j1 = (int)(e / p2), r = (int)(e % p2);
            double v = 0.0;
            for (int m1 = 0; m1 < n; ++m1) {
                const double er = E[2 * (m1 * p + j1)], ei = E[2 * (m1 * p + j1) + 1];
                v += er * S[R.C2r + m1 * p2 + r] + ei * S[R.C2i + m1 * p2 + r];
            }
            D.w0vals[(int64_t)b * p3 + e] = (T)v;
        }
        break;
    }
}

int64_t root_scratch_elems(const Tables &t, int npts)
{
    return RootLayout(t.p, t.nwn, t.nwh, npts).total;
}

// -------------------------------------------------------------- small ones
__global__ void k_gather_q(const double *charges, const int32_t *perm, int64_t n, double *qs)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) qs[i] = charges[perm[i]];
}

// scale[b]: the unit change of problem b, whose points are [poff[b], poff[b+1]) in tree order
__global__ void k_finalize(const double *ufar, const double *ures, const int32_t *perm, int64_t n, const double *scale,
                           const int64_t *poff, int nprob, double *pot, double *farp, double *nearp)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nprob - 1;  // the problem b with poff[b] <= i < poff[b+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (poff[mid] <= i) lo = mid; else hi = mid - 1;
    }
    int64_t j = perm[i];
    double f = ufar[i] * scale[lo], r = ures[i] * scale[lo];
    if (pot) pot[j] = f + r;
    if (farp) farp[j] = f;
    if (nearp) nearp[j] = r;
}

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

// Leaf targets of the FP32 path on matrix cores: per anchor, 16 targets per
// wave at a time.  W((j1 j2), t) = sum_j3 v[(j1 j2)][j3] Lz_t[j3] is an MFMA
// mode product (rows (j1 j2), columns the targets); each lane then folds its
// four rows of W with Lx_t[j1] Ly_t[j2] and the four lanes of a target add up.
template <typename T, int P>
__global__ void __launch_bounds__(TPB) k_leaf_mfma(Dev<T> D, const int32_t *anc, const int32_t *tbeg,
                                                   const int32_t *tgt)
{
    constexpr int P2 = P * P, P3 = P2 * P, NSL = (P2 + 15) / 16, NKS = (P + 3) / 4;
    __shared__ T v[P3], xc[P], bw[P];
    __shared__ T Lr[NWAVE][3][16][P];  // Lagrange rows x, y, z of the wave's 16 targets
    const int a = blockIdx.x;
    const int b0 = tbeg[a], b1 = tbeg[a + 1];
    if (b0 == b1) return;  // whole block
    const int32_t A = anc[a];
    const T *src = D.local + (int64_t)a * P3;
    for (int t = threadIdx.x; t < P3; t += TPB) v[t] = src[t];
    for (int t = threadIdx.x; t < P; t += TPB) { xc[t] = D.xcheb[t]; bw[t] = D.bary[t]; }
    const double cA[3] = {D.bcenter[3 * (int64_t)A], D.bcenter[3 * (int64_t)A + 1], D.bcenter[3 * (int64_t)A + 2]};
    const double sc = 2.0 / box_side(D.blevel[A]);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, kq = l >> 4, r16 = l & 15;
    __syncthreads();
    // each wave takes its own groups of 16 targets (the Lagrange rows in LDS
    // are per wave, so no block barrier is needed past the set-up), and a
    // wave with no targets left stops instead of running empty products
    for (int base = b0 + 16 * w; base < b1; base += 16 * NWAVE) {
        const int t = base + r16;
        const bool tv = t < b1;
        if (kq < 3) {
            T row[P];
            if (tv) {
                const int64_t i = tgt[t];
                const double x = (kq == 0) ? D.Xt[i] : (kq == 1) ? D.Yt[i] : D.Zt[i];
                lagrange_row_fast<T, P>(xc, bw, (T)((x - cA[kq]) * sc), row);
            } else {
#pragma unroll
                for (int j = 0; j < P; ++j) row[j] = T(0);
            }
#pragma unroll
            for (int j = 0; j < P; ++j) Lr[w][kq][r16][j] = row[j];
        }
        // the wave's LDS writes above precede its reads below (one wave's LDS
        // operations complete in order; this keeps the compiler from moving them)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        T bz[NKS];
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int k = 4 * s + kq;
            bz[s] = (k < P) ? Lr[w][2][r16][k] : T(0);
        }
        T part = T(0);
        // LU slabs at a time (independent MFMA chains); the lane's first row
        // x0 = 16 sl + RB kq is tracked as (x0 / P, x0 % P), its rows are
        // x0 + RS q
        constexpr int LU = 3, RB = Mfma<T>::RB, RS = Mfma<T>::RS;
        int i0 = (RB * kq) / P, i1 = (RB * kq) % P;
#pragma unroll 1
        for (int sl = 0; sl < NSL; sl += LU) {
            v4_t<T> acc[LU];
#pragma unroll
            for (int u = 0; u < LU; ++u) acc[u] = v4_t<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                const int k = 4 * s + kq;
#pragma unroll
                for (int u = 0; u < LU; ++u) {
                    const int xa = 16 * (sl + u) + r16;
                    const T av = (xa < P2 && k < P) ? v[xa * P + k] : T(0);
                    acc[u] = Mfma<T>::mma(av, bz[s], acc[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < LU; ++u) {
                const int x0 = 16 * (sl + u) + RB * kq;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int j0 = i0, j1 = i1 + RS * q;
                    if constexpr (RS == 1) {
                        if (j1 >= P) { j1 -= P; ++j0; }
                    } else {
                        while (j1 >= P) { j1 -= P; ++j0; }
                    }
                    if (x0 + RS * q < P2) part += Lr[w][0][r16][j0] * Lr[w][1][r16][j1] * acc[u][q];
                }
                // next slab: x0 += 16
                i1 += 16;
                while (i1 >= P) { i1 -= P; ++i0; }
            }
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (kq == 0 && tv) D.ufar[tgt[t]] = (double)part;
        // this round's reads of Lr[w] precede the next round's writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ------------------------------------------------------------ host side
template <typename T, int P, int NF>
struct Cfg {
    static constexpr int P2 = P * P, P3 = P2 * P, NN = 2 * NF + 1, NH = NF + 1;
    static size_t lds_up() { return sizeof(T) * (2 * P2 + 2 * P + up_work<T, P>()); }
};

template <typename T>
Dev<T> make_dev(Plan *P)
{
    Dev<T> D;
    const Tables &t = P->tab;
    D.p = t.p; D.nf = t.nf; D.nn = t.nn; D.nh = t.nh; D.nw = t.nw; D.nwn = t.nwn; D.nwh = t.nwh;
    D.gdeg = sizeof(T) == 8 ? t.gdeg : t.gdeg32;
    D.X = P->Xs; D.Y = P->Ys; D.Z = P->Zs; D.qs = P->qs;
    D.Xt = P->Xt; D.Yt = P->Yt; D.Zt = P->Zt; D.tstart = P->tstart; D.tcount = P->tcount;
    D.pstart = P->sstart; D.pcount = P->scount; D.child0 = P->child0; D.parent = P->parent; D.col = P->colleague;
    D.proxy_slot = P->proxy_slot; D.local_slot = P->local_slot; D.psi_slot = P->psi_slot; D.blevel = P->blevel;
    D.anchor = P->anchor;
    D.anc_read = P->anc_read;
    D.bflags = P->bflags; D.bcenter = P->bcenter;
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
    D.ufar = P->ufar; D.ures = P->ures; D.rootscratch = P->rootscratch;
    D.pwstride = pw_stride(t);
    D.ywd = nullptr;
    D.ycheb = nullptr;
    D.yself = nullptr;
    D.ywd_stride = 0;
    D.ylam = 0.0;
    D.ydeg = 0;
    D.ynlev = 0;
    D.wshift = (t.kind == 2) ? 2 : 1;
    D.root_npmax = (int)std::min<int64_t>(P->n, P->leaf_max);
    D.root_stride = root_scratch_elems(t, D.root_npmax);
    if (P->kernel == DMK_YUKAWA && P->dim == 3) {
        D.ywd = (const T *)(f64 ? (void *)P->y_wd64 : (void *)P->y_wd32);
        D.ycheb = (const T *)(f64 ? (void *)P->y_cheb64 : (void *)P->y_cheb32);
        D.yself = P->y_self;
        D.ywd_stride = (int64_t)t.nh * t.nn * t.nn;
        D.ylam = P->lambda * P->pside[0];
        D.ydeg = f64 ? P->y_deg : P->y_deg32;
        D.ynlev = P->nlevels;
    }
    return D;
}

template <typename K>
void allow_lds(K kernel, size_t bytes)
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

// residual sums with the polynomial degree rounded up to a compiled bucket
// the residual kernel for the series degree (a compile-time bucket)
template <typename T, int POW>
static void launch_residual_deg(const Dev<T> &D, Plan *Pl, dim3 g, dim3 b, size_t lds, hipStream_t s)
{
    if (D.gdeg <= 7)
        hipLaunchKernelGGL((k_residual<T, 7, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else if (D.gdeg <= 9)
        hipLaunchKernelGGL((k_residual<T, 9, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else if (D.gdeg <= 11)
        hipLaunchKernelGGL((k_residual<T, 11, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else if (D.gdeg <= 13)
        hipLaunchKernelGGL((k_residual<T, 13, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else if (D.gdeg <= 15)
        hipLaunchKernelGGL((k_residual<T, 15, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else if (D.gdeg <= 20)
        hipLaunchKernelGGL((k_residual<T, 20, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
    else
        hipLaunchKernelGGL((k_residual<T, 47, POW>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
}

template <typename T>
static void launch_residual(const Dev<T> &D, Plan *Pl, hipStream_t s)
{
    const dim3 g((unsigned)Pl->nleaf), b(TPB);
    const size_t lds = sizeof(int32_t) * 3 * ((size_t)Pl->nl_max + 1);  // loff, and (k_residual) lbeg, llev
    if (D.ywd) {
        hipLaunchKernelGGL((k_residual_y3<T>), g, b, lds, s, D, Pl->l_leaf, Pl->nl_off, Pl->nl_src, Pl->nl_pre);
        return;
    }
    if (D.wshift == 2)
        launch_residual_deg<T, 2>(D, Pl, g, b, lds, s);
    else
        launch_residual_deg<T, 1>(D, Pl, g, b, lds, s);
}

// persistent grids of the queue-fed kernels (set with the LDS limits, before
// any graph capture)
template <typename T, int P, int NF>
struct QGrid {
    static inline unsigned upward = 0;
};

// dynamic LDS limits of the stage kernels, once per process
template <typename T, int P, int NF>
static void set_lds_attrs()
{
    using C = Cfg<T, P, NF>;
    static bool attrs = false;
    if (attrs) return;
    allow_lds(k_upward<T, P>, C::lds_up());
    allow_lds(k_upward_q<T, P>, C::lds_up());
    const size_t lds_mfma = LocalMfma<T, P, NF>::lds();
    allow_lds(k_local_mfma<T, P, NF>, lds_mfma);
    allow_lds(k_local_mfma_q<T, P, NF>, lds_mfma);
    allow_lds(k_proxy2pw_mfma<T, P, NF>, P2pwMfma<T, P, NF>::lds());
    (void)queue_wait_ticks();
    QGrid<T, P, NF>::upward = resident_blocks(k_upward_q<T, P>, TPB, C::lds_up());
    attrs = true;
}


// Root window W_0, outgoing and incoming plane waves and the local values of
// the anchors: the stages between the proxy charges and the evaluation at
// the targets, shared by the point code and the volume code.
template <typename T, int P, int NF>
static void enqueue_far(Plan *Pl, hipStream_t s)
{
    using C = Cfg<T, P, NF>;
    Dev<T> D = make_dev<T>(Pl);
    const auto &ll = Pl->ll;
    const int L = Pl->nlevels;
    const int64_t n = Pl->n;
    {
        StageScope t(Pl, s, DMK_STAGE_ROOT);
        // every problem's root at once (grid y); stage 0 only if some root is a leaf
        const bool any_leaf_root = ll.fout_off[1] < Pl->nprob;
        const int64_t p = P, nw = Pl->tab.nwn, nwh = Pl->tab.nwh;
        const int64_t outs[8] = {3 * (int64_t)D.root_npmax, p * p * p, p * p * nwh, p * nwh * nw, nw * nwh * nw,
                                 nw * nw * p, nw * p * p, p * p * p};
        for (int st = any_leaf_root ? 0 : 1; st < 8; ++st)
            hipLaunchKernelGGL((k_root_stage<T>), dim3(nblk(outs[st]), (unsigned)Pl->nprob), dim3(TPB), 0, s, D, st);
    }
    // Step 3: outgoing plane waves of every F_out box and incoming plane
    // waves of every non-empty F_in box, all levels in one launch each
    if (Pl->nfout) {
        StageScope t(Pl, s, DMK_STAGE_PROXY2PW);
        hipLaunchKernelGGL((k_proxy2pw_mfma<T, P, NF>), dim3((unsigned)Pl->nfout), dim3(P2PW_NT),
                           (P2pwMfma<T, P, NF>::lds()), s, D, Pl->l_fout);
    }
    if (Pl->noct) {
        StageScope t(Pl, s, DMK_STAGE_PWSHIFT);
        const int64_t nmode = (int64_t)Pl->tab.nh * Pl->tab.nn * Pl->tab.nn;
        const int nchunk = (int)((nmode + TPB - 1) / TPB);
        constexpr int RB = sizeof(T) == 4 ? 2 : 1;  // source rows per batch of loads
        const int64_t nb = 8 * ((Pl->noct + 7) / 8) * nchunk;
        hipLaunchKernelGGL((k_pwshift<T, RB>), dim3((unsigned)nb), dim3(TPB), 0, s, D, Pl->oct_dst, Pl->oct_src,
                           Pl->oct_level, Pl->noct, nchunk);
    }
    // local values of the anchors, coarse to fine: one queue-fed launch over
    // all levels, or one launch per level
    if (Pl->nanc && Pl->queued) {
        StageScope t(Pl, s, DMK_STAGE_PW2GRID);
        const WorkQ q = local_queue(Pl);
        reset_queue(q.head, 4 + Pl->nanc, s);
        hipLaunchKernelGGL((k_local_mfma_q<T, P, NF>), dim3((unsigned)Pl->nanc), dim3(LOCAL_NT),
                           (LocalMfma<T, P, NF>::lds()), s, D, q);
        return;
    }
    for (int l = 0; l < L; ++l) {
        int64_t nan = ll.anc_off[l + 1] - ll.anc_off[l];
        if (!nan) continue;
        StageScope t(Pl, s, DMK_STAGE_PW2GRID);
        hipLaunchKernelGGL((k_local_mfma<T, P, NF>), dim3((unsigned)nan), dim3(LOCAL_NT), (LocalMfma<T, P, NF>::lds()),
                           s, D, Pl->l_anc + ll.anc_off[l], l);
    }
}

// The far-field chain between the charge gather and the final scatter
// (upward pass to leaf evaluation).  It reads and writes plan-owned buffers
// only, so it can be captured into a HIP graph once and replayed.  The
// residual sums are not part of it: they depend on the gathered charges only
// and run beside the chain (run_eval_t).
template <typename T, int P, int NF>
static void enqueue_chain(Plan *Pl, hipStream_t s)
{
    using C = Cfg<T, P, NF>;
    Dev<T> D = make_dev<T>(Pl);
    const auto &ll = Pl->ll;
    const int L = Pl->nlevels;
    // Step 2: upward pass, finest level first: one queue-fed launch over all
    // levels, or one launch per level
    if (Pl->nfout && Pl->queued) {
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        const WorkQ q = upward_queue(Pl);
        reset_queue(q.head, 4 + Pl->nfout, s);
        hipLaunchKernelGGL((k_upward_q<T, P>), dim3((unsigned)std::min<int64_t>(Pl->nfout, QGrid<T, P, NF>::upward)),
                           dim3(TPB),
                           C::lds_up(), s, D, q);
    }
    for (int l = L - 1; l >= 0 && !Pl->queued; --l) {
        int64_t m = ll.fout_off[l + 1] - ll.fout_off[l];
        if (!m) continue;
        StageScope t(Pl, s, DMK_STAGE_UPWARD);
        hipLaunchKernelGGL((k_upward<T, P>), dim3((unsigned)m), dim3(TPB), C::lds_up(), s, D, Pl->l_fout + ll.fout_off[l]);
    }
    enqueue_far<T, P, NF>(Pl, s);
    if (Pl->nleaf) {
        StageScope t(Pl, s, DMK_STAGE_LEAF);
        hipLaunchKernelGGL((k_leaf_mfma<T, P>), dim3((unsigned)Pl->nanc), dim3(TPB), 0, s, D, Pl->l_anc, Pl->anc_tbeg,
                           Pl->anc_tgt);
    }
}

template <typename T, int P, int NF>
static void run_eval_t(Plan *Pl, const double *charges, double *pot, double *far_part, double *near_part,
                       hipStream_t s)
{
    using C = Cfg<T, P, NF>;
    const int64_t n = Pl->n;
    set_lds_attrs<T, P, NF>();
    {
        StageScope t(Pl, s, DMK_STAGE_GATHER);
        hipLaunchKernelGGL(k_gather_q, dim3(nblk(Pl->nsrc)), dim3(TPB), 0, s, charges, Pl->sperm, Pl->nsrc, Pl->qs);
    }
    const bool batched = (Pl->flags & DMK_FLAG_BATCHED) && !Pl->timing;
    if (batched) {
        // the residual sums on the side stream, beside the replayed chain: a
        // second hardware queue lets their workgroups fill the room the
        // chain's memory-bound stages leave (measured: a graph holding both
        // branches ran them with less overlap)
        if (Pl->nleaf) {
            DMK_HIP(hipEventRecord(Pl->ev_fork, s));
            DMK_HIP(hipStreamWaitEvent(Pl->side_stream, Pl->ev_fork, 0));
            launch_residual<T>(make_dev<T>(Pl), Pl, Pl->side_stream);
            DMK_HIP(hipEventRecord(Pl->ev_join, Pl->side_stream));
        }
        if (!Pl->graph_exec) {
            // capture once: the chain touches plan-owned buffers only
            hipGraph_t g = nullptr;
            DMK_HIP(hipStreamBeginCapture(Pl->cap_stream, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_chain<T, P, NF>(Pl, Pl->cap_stream);
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
        if (Pl->nleaf) DMK_HIP(hipStreamWaitEvent(s, Pl->ev_join, 0));
    } else {
        enqueue_chain<T, P, NF>(Pl, s);
        if (Pl->nleaf) {
            StageScope t(Pl, s, DMK_STAGE_RESIDUAL);
            launch_residual<T>(make_dev<T>(Pl), Pl, s);
        }
    }
    {
        StageScope t(Pl, s, DMK_STAGE_FINALIZE);
        hipLaunchKernelGGL(k_finalize, dim3(nblk(Pl->ntgt)), dim3(TPB), 0, s, Pl->ufar, Pl->ures, Pl->tperm, Pl->ntgt,
                           (const double *)Pl->d_pscale, (const int64_t *)Pl->d_poff, Pl->nprob, pot, far_part,
                           near_part);
    }
    DMK_HIP(hipGetLastError());
}

void far_stages(Plan *P, hipStream_t s)
{
    if (P->dim != 3 || P->p != 18) throw Error{DMK_ERR_UNSUPPORTED, "far-field stages are built for p = 18 in 3-D"};
    if (P->precision == DMK_FP64) {
        set_lds_attrs<double, 18, 12>();
        enqueue_far<double, 18, 12>(P, s);
    } else {
        set_lds_attrs<float, 18, 12>();
        enqueue_far<float, 18, 12>(P, s);
    }
}

void run_eval(Plan *P, const double *charges, double *pot, double *far_part, double *near_part, hipStream_t s)
{
    if (P->n == 0) return;
    if (!P->qs)
        throw Error{DMK_ERR_STATE, "the plan holds no eval workspace (DMK_FLAG_NO_WORKSPACE): use dmk_eval_noalloc"};
    if (P->dim == 2) {
        run_eval2(P, charges, pot, far_part, near_part, s);
        return;
    }
    const bool f64 = P->precision == DMK_FP64;
    switch (P->p) {
    case 18:
        if (f64) run_eval_t<double, 18, 12>(P, charges, pot, far_part, near_part, s);
        else run_eval_t<float, 18, 12>(P, charges, pot, far_part, near_part, s);
        break;
    case 15:
        if (f64) run_eval_t<double, 15, 10>(P, charges, pot, far_part, near_part, s);
        else run_eval_t<float, 15, 10>(P, charges, pot, far_part, near_part, s);
        break;
    case 9:
        if (f64) run_eval_t<double, 9, 6>(P, charges, pot, far_part, near_part, s);
        else run_eval_t<float, 9, 6>(P, charges, pot, far_part, near_part, s);
        break;
    default:
        throw Error{DMK_ERR_UNSUPPORTED, "no kernels for this proxy order"};
    }
}


// coefficients a_k of sum_k c_k T_k(u) = sum_k a_k u^k for k <= deg
static std::vector<double> cheb_to_power(const std::vector<double> &c, int deg)
{
    if (c.empty()) return std::vector<double>(1, 0.0);  // no residual series (volume plans)
    deg = std::max(0, std::min(deg, (int)c.size() - 1));
    std::vector<double> a(deg + 1, 0.0), tm(deg + 1, 0.0), tk(deg + 1, 0.0), tp(deg + 1, 0.0);
    tm[0] = 1.0;  // T_0
    a[0] = c[0];
    if (deg >= 1) {
        tk[1] = 1.0;  // T_1 = u
        a[1] += c[1];
    }
    for (int k = 1; k < deg; ++k) {
        // T_{k+1} = 2u T_k - T_{k-1}
        for (int i = 0; i <= deg; ++i) tp[i] = (i > 0 ? 2.0 * tk[i - 1] : 0.0) - tm[i];
        for (int i = 0; i <= deg; ++i) a[i] += c[k + 1] * tp[i];
        tm.swap(tk);
        tk.swap(tp);
    }
    return a;
}

void upload_tables(Plan *P, hipStream_t s)
{
    const Tables &t = P->tab;
    auto up = [&](const std::vector<double> &v) {
        double *d = (double *)dalloc(P, std::max<size_t>(v.size(), 1) * sizeof(double));
        if (!v.empty()) DMK_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
        return d;
    };
    std::vector<std::vector<float>> keep;
    auto upf = [&](const std::vector<double> &v) {
        keep.emplace_back(v.begin(), v.end());
        const auto &h = keep.back();
        float *d = (float *)dalloc(P, std::max<size_t>(h.size(), 1) * sizeof(float));
        if (!h.empty()) DMK_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s));
        return d;
    };
    P->d_c2p = up(t.c2p);
    P->d_epw = up(t.epw);
    P->d_ew = up(t.ew);
    P->d_wd0 = up(t.wd0);
    P->d_ww = up(t.ww);
    std::vector<double> gpad(t.gcheb);
    gpad.resize(std::max<size_t>(gpad.size(), 48), 0.0);  // room for a fixed number of terms
    P->d_gcheb = up(gpad);
    // power-series coefficients in u of the series truncated at the FP64 and
    // the FP32 degree (the residual kernels evaluate them by Horner's rule)
    std::vector<double> gm64 = cheb_to_power(t.gcheb, t.gdeg), gm32 = cheb_to_power(t.gcheb, t.gdeg32);
    gm64.resize(48, 0.0);
    gm32.resize(48, 0.0);
    P->d_gmono = up(gm64);
    P->f_gmono = upf(gm32);
    P->d_xcheb = up(t.xcheb);
    P->d_bary = up(t.bary);
    P->f_c2p = upf(t.c2p);
    P->f_epw = upf(t.epw);
    P->f_wd0 = upf(t.wd0);
    P->f_gcheb = upf(gpad);
    P->f_xcheb = upf(t.xcheb);
    P->f_bary = upf(t.bary);
    DMK_HIP(hipStreamSynchronize(s));
}

// The eval workspace of a point plan: buffers every eval writes before it
// reads them (gathered charges, proxies, plane waves, local values, partial
// potentials, root scratch).  Listed once, for alloc_workspace and for the
// static-scratch eval.
void workspace_layout(Plan *P, std::vector<WsItem> &items)
{
    if (P->dim == 2) {
        workspace_layout2(P, items);
        return;
    }
    const Tables &t = P->tab;
    const size_t el = (P->precision == DMK_FP64) ? sizeof(double) : sizeof(float);
    const int64_t p3 = (int64_t)t.p * t.p * t.p;
    const int64_t nm = pw_stride(t);
    auto add = [&](void *field, int64_t cnt, size_t sz) {
        items.push_back({(void **)field, (size_t)std::max<int64_t>(cnt, 1) * sz});
    };
    add(&P->qs, P->nsrc, 8);
    add(&P->ufar, P->ntgt, 8);
    add(&P->ures, P->ntgt, 8);
    add(&P->rootscratch, P->nprob * root_scratch_elems(t, (int)std::min<int64_t>(P->n, P->leaf_max)), 8);
    add(&P->proxy, P->nfout * p3, el);
    add(&P->local, P->nanc * p3, el);
    add(&P->phi, 2 * P->nfout * nm, el);
    add(&P->psi, 2 * P->nfin * nm, el);
    add(&P->w0vals, P->nprob * p3, el);
    add(&P->qctl, queue_ctl_words(P), 4);
}

void alloc_workspace(Plan *P)
{
    std::vector<WsItem> items;
    workspace_layout(P, items);
    P->ws_bytes = 0;
    for (const WsItem &it : items) P->ws_bytes += (int64_t)((it.bytes + 255) / 256 * 256);
    if ((P->flags & DMK_FLAG_NO_WORKSPACE) && !P->is_vol) return;  // evaluated from the static scratch
    for (const WsItem &it : items) *it.ptr = dalloc(P, it.bytes);
    P->has_workspace = true;
}

// ---------------------------------------------------------- work counts
namespace {
// pairs of the residual lists closer than the source box side (r < s_l)
// targets: Xt.. with tstart/tcount; sources: X.. with pstart/pcount
__global__ void __launch_bounds__(TPB) k_count_inrange(const double *X, const double *Y, const double *Z,
                                                       const int32_t *pstart, const int32_t *pcount,
                                                       const double *Xt, const double *Yt, const double *Zt,
                                                       const int32_t *tstart, const int32_t *tcount,
                                                       const int32_t *leaves, const int32_t *nl_off,
                                                       const int32_t *nl_src, const int32_t *blevel,
                                                       unsigned long long *total)
{
    __shared__ unsigned long long red[TPB];
    const int32_t B = leaves[blockIdx.x];
    const int64_t t0 = tstart[B];
    const int nt = tcount[B];
    unsigned long long cnt = 0;
    for (int tt = threadIdx.x; tt < nt; tt += TPB) {
        const double xt = Xt[t0 + tt], yt = Yt[t0 + tt], zt = Zt ? Zt[t0 + tt] : 0.0;
        for (int li = nl_off[blockIdx.x]; li < nl_off[blockIdx.x + 1]; ++li) {
            const int32_t T = nl_src[li];
            const double s = ldexp(1.0, -blevel[T]), s2 = s * s;
            for (int64_t j = pstart[T]; j < pstart[T] + pcount[T]; ++j) {
                double dx = xt - X[j], dy = yt - Y[j], dz = Z ? zt - Z[j] : 0.0;
                cnt += (dx * dx + dy * dy + dz * dz < s2) ? 1 : 0;
            }
        }
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, red[0]);
}
}  // namespace

void count_work(Plan *P, hipStream_t s)
{
    const int64_t nb = P->nbox;
    const int NC = 1 << P->dim, NCOL = (P->dim == 3) ? 27 : 9;
    std::vector<uint8_t> fl(nb);
    std::vector<int32_t> pc(nb), tc(nb), c0(nb), col;  // sources and targets per box
    DMK_HIP(hipMemcpy(fl.data(), P->bflags, nb, hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(pc.data(), P->scount, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(tc.data(), P->tcount, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    DMK_HIP(hipMemcpy(c0.data(), P->child0, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    col.resize((size_t)nb * NCOL);
    DMK_HIP(hipMemcpy(col.data(), P->colleague, (size_t)nb * NCOL * sizeof(int32_t), hipMemcpyDeviceToHost));
    P->n_anterp = P->n_merge = P->n_shift_pairs = 0;
    for (int r = 0; r < P->nprob && r < nb; ++r)
        if (!(fl[r] & 2)) P->n_anterp += pc[r];  // a root leaf is anterpolated in the root stage
    for (int64_t b = 0; b < nb; ++b) {
        if (fl[b] & 2)
            for (int k = 0; k < NC; ++k) {
                int32_t c = c0[b] + k;
                if (pc[c] == 0) continue;
                if (fl[c] & 2) P->n_merge++; else P->n_anterp += pc[c];
            }
        if ((fl[b] & 4) && tc[b] > 0)
            for (int k = 0; k < NCOL; ++k) {
                int32_t j = col[(size_t)b * NCOL + k];
                if (j >= 0 && (fl[j] & 2)) P->n_shift_pairs++;
            }
    }
    P->nanc_tgt = 0;
    if (P->nanc) {
        std::vector<int32_t> tb(P->nanc + 1);
        DMK_HIP(hipMemcpy(tb.data(), P->anc_tbeg, (P->nanc + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t a = 0; a < P->nanc; ++a) P->nanc_tgt += (tb[a + 1] > tb[a]);
    }
    P->npairs_in = 0;
    if (P->nleaf) {
        unsigned long long *d = nullptr;
        DMK_HIP(hipMalloc(&d, sizeof(unsigned long long)));
        DMK_HIP(hipMemsetAsync(d, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_count_inrange, dim3((unsigned)P->nleaf), dim3(TPB), 0, s, P->Xs, P->Ys, P->Zs, P->sstart,
                           P->scount, P->Xt, P->Yt, P->Zt, P->tstart, P->tcount, P->l_leaf, P->nl_off, P->nl_src,
                           P->blevel, d);
        unsigned long long h = 0;
        DMK_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        DMK_HIP(hipFree(d));
        P->npairs_in = (int64_t)h;
    }
}

// Algorithmic work of one eval: flops of the separable contractions and
// pair evaluations, and the bytes that must cross HBM once.
void stage_work(const Plan *P, double *F, double *Bt)
{
    const Tables &t = P->tab;
    const double el = (P->precision == DMK_FP64) ? 8.0 : 4.0;
    const double p = t.p, n = t.nn, nh = t.nh;
    const double N = (double)P->ntgt, Ns = (double)P->nsrc;  // targets, sources
    for (int i = 0; i < DMK_NSTAGES; ++i) F[i] = Bt[i] = 0.0;
    Bt[DMK_STAGE_GATHER] = 20 * Ns;
    Bt[DMK_STAGE_FINALIZE] = 28 * N;
    const double gd = (double)((P->precision == DMK_FP64) ? t.gdeg : t.gdeg32);
    if (P->dim == 2) {
        const double p2 = p * p, p3 = p2 * p;
        const double pwflops = 4 * nh * p2 + 8 * nh * n * p;  // one box, either direction
        const double pwbytes = 2 * el * nh * n;
        F[DMK_STAGE_UPWARD] = 2 * p2 * P->n_anterp + 4 * p3 * P->n_merge;
        Bt[DMK_STAGE_UPWARD] = 24.0 * P->n_anterp + el * p2 * (P->n_merge + P->nfout);
        const double nw = t.nwn, nwh = t.nwh;
        F[DMK_STAGE_ROOT] = P->nprob * 2 * (4 * nwh * p2 + 8 * nwh * nw * p);
        Bt[DMK_STAGE_ROOT] = 16 * p2 * P->nprob;
        F[DMK_STAGE_PROXY2PW] = pwflops * P->nfout;
        Bt[DMK_STAGE_PROXY2PW] = (el * p2 + pwbytes) * P->nfout;
        F[DMK_STAGE_PWSHIFT] = 8 * nh * n * P->n_shift_pairs;
        Bt[DMK_STAGE_PWSHIFT] = pwbytes * (P->nfout + P->nfin);
        F[DMK_STAGE_PW2GRID] = pwflops * P->nfin + 4 * p3 * std::max<int64_t>(P->nanc - P->nprob, 0);
        Bt[DMK_STAGE_PW2GRID] = pwbytes * P->nfin + 2 * el * p2 * P->nanc;
        F[DMK_STAGE_LEAF] = 2 * p2 * N;
        Bt[DMK_STAGE_LEAF] = 32 * N + el * p2 * P->nanc_tgt;  // one block per anchor reads its values once
        F[DMK_STAGE_RESIDUAL] = 6.0 * P->npairs + (2.0 * gd + 12.0) * P->npairs_in;
        Bt[DMK_STAGE_RESIDUAL] = 32 * N;
        return;
    }
    if (P->is_vol) {
        vol_stage_work(P, F, Bt);
        return;
    }
    const double p3 = p * p * p, p4 = p3 * p;
    const double pwflops = 4 * nh * p3 + 8 * nh * n * p * p + 8 * nh * n * n * p;  // one box, either direction
    const double pwbytes = 2 * el * nh * n * n;                                      // one half spectrum
    F[DMK_STAGE_UPWARD] = 2 * p3 * P->n_anterp + 6 * p4 * P->n_merge;
    Bt[DMK_STAGE_UPWARD] = 32.0 * P->n_anterp + el * p3 * (P->n_merge + P->nfout);
    {
        const double nw = t.nwn, nwh = t.nwh;
        F[DMK_STAGE_ROOT] = 2 * (4 * nwh * p3 + 8 * nwh * nw * p * p + 8 * nwh * nw * nw * p);
        Bt[DMK_STAGE_ROOT] = 16 * p3;
    }
    F[DMK_STAGE_PROXY2PW] = pwflops * P->nfout;
    Bt[DMK_STAGE_PROXY2PW] = (el * p3 + pwbytes) * P->nfout;
    F[DMK_STAGE_PWSHIFT] = 8 * nh * n * n * P->n_shift_pairs;
    Bt[DMK_STAGE_PWSHIFT] = pwbytes * (P->nfout + P->nfin);
    // anchors: interpolation from the anchor ancestor (6 p^4) plus the plane waves
    F[DMK_STAGE_PW2GRID] = pwflops * P->nfin + 6 * p4 * std::max<int64_t>(P->nanc - 1, 0);
    Bt[DMK_STAGE_PW2GRID] = pwbytes * P->nfin + 2 * el * p3 * P->nanc;
    F[DMK_STAGE_LEAF] = 2 * p3 * N;
    Bt[DMK_STAGE_LEAF] = 40 * N + el * p3 * P->nanc_tgt;  // one block per anchor reads its values once
    F[DMK_STAGE_RESIDUAL] = 8.0 * P->npairs + (2.0 * gd + 8.0) * P->npairs_in;
    if (P->kernel == DMK_YUKAWA) {  // Clenshaw (4 flop per term), exp and a division per pair in range
        const double yd = (double)((P->precision == DMK_FP64) ? P->y_deg : P->y_deg32);
        F[DMK_STAGE_RESIDUAL] = 8.0 * P->npairs + (4.0 * yd + 16.0) * P->npairs_in;
    }
    Bt[DMK_STAGE_RESIDUAL] = 40 * N;
}

}  // namespace dmk
