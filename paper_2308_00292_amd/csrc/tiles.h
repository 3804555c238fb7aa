// Device helpers shared by the kernels of the point code (eval.hip) and of the
// volume code (vol.hip): register-tiled small GEMMs on LDS operands, tile
// shapes per Chebyshev order, and the barycentric Lagrange basis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmk {
namespace {

constexpr int TPB = 256;

// --------------------------------------------------------------- GEMM
// C(b,m,n) = [C(b,m,n) +] sum_k A(b,m,k) B(b,k,n), all operands addressed by
// strides.  Each thread owns a TM x TN tile whose rows are MT apart and whose
// columns are NT apart (MT, NT = number of tiles along m, n), so consecutive
// threads read consecutive columns of B and share rows of A.
template <typename T, int TM, int TN, bool ACC>
__device__ inline void gemm(int nb, int M, int N, int K, const T *A, int sAb, int sAm, int sAk, const T *B,
                            int sBb, int sBk, int sBn, T *C, int sCb, int sCm, int sCn)
{
    const int MT = (M + TM - 1) / TM, NT = (N + TN - 1) / TN;
    const int ntile = nb * MT * NT;
    for (int t = threadIdx.x; t < ntile; t += TPB) {
        const int b = t / (MT * NT), r = t % (MT * NT);
        const int mt = r / NT, nt = r % NT;
        const T *Ab = A + (int64_t)b * sAb;
        const T *Bb = B + (int64_t)b * sBb;
        T acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = T(0);
        for (int k = 0; k < K; ++k) {
            T a[TM], bb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                int m = mt + i * MT;
                a[i] = (m < M) ? Ab[m * sAm + k * sAk] : T(0);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                int n = nt + j * NT;
                bb[j] = (n < N) ? Bb[k * sBk + n * sBn] : T(0);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] += a[i] * bb[j];
        }
        T *Cb = C + (int64_t)b * sCb;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                int m = mt + i * MT, n = nt + j * NT;
                if (m < M && n < N) {
                    if (ACC) Cb[m * sCm + n * sCn] += acc[i][j];
                    else Cb[m * sCm + n * sCn] = acc[i][j];
                }
            }
    }
}

// Same contraction with the output kept in registers: acc[i][j] holds
// C(m = mt + i MT, n = nt + j NT) of the thread's single tile (requires
// MT * NT <= TPB).  Used for the per-box accumulators of shape p x p^2.
template <typename T, int TM, int TN>
__device__ inline void gemm_regs(int M, int N, int K, const T *A, int sAm, int sAk, const T *B, int sBk, int sBn,
                                 T (&acc)[TM][TN])
{
    const int MT = (M + TM - 1) / TM, NT = (N + TN - 1) / TN;
    const int t = threadIdx.x;
    if (t >= MT * NT) return;
    const int mt = t / NT, nt = t % NT;
    for (int k = 0; k < K; ++k) {
        T a[TM], bb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            int m = mt + i * MT;
            a[i] = (m < M) ? A[m * sAm + k * sAk] : T(0);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            int n = nt + j * NT;
            bb[j] = (n < N) ? B[k * sBk + n * sBn] : T(0);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] += a[i] * bb[j];
    }
}

// Complex contraction on planar operands (real and imaginary parts at
// separate base pointers with identical strides).
template <typename T, int TM, int TN, bool ACC>
__device__ inline void cgemm(int nb, int M, int N, int K, const T *Ar, const T *Ai, int sAb, int sAm, int sAk,
                             const T *Br, const T *Bi, int sBb, int sBk, int sBn, T *Cr, T *Ci, int sCb, int sCm,
                             int sCn)
{
    const int MT = (M + TM - 1) / TM, NT = (N + TN - 1) / TN;
    const int ntile = nb * MT * NT;
    for (int t = threadIdx.x; t < ntile; t += TPB) {
        const int b = t / (MT * NT), r = t % (MT * NT);
        const int mt = r / NT, nt = r % NT;
        const int64_t oA = (int64_t)b * sAb, oB = (int64_t)b * sBb;
        T re[TM][TN], im[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) re[i][j] = im[i][j] = T(0);
        for (int k = 0; k < K; ++k) {
            T ar[TM], ai[TM], br[TN], bi[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                int m = mt + i * MT;
                bool ok = m < M;
                ar[i] = ok ? Ar[oA + m * sAm + k * sAk] : T(0);
                ai[i] = ok ? Ai[oA + m * sAm + k * sAk] : T(0);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                int n = nt + j * NT;
                bool ok = n < N;
                br[j] = ok ? Br[oB + k * sBk + n * sBn] : T(0);
                bi[j] = ok ? Bi[oB + k * sBk + n * sBn] : T(0);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    re[i][j] += ar[i] * br[j] - ai[i] * bi[j];
                    im[i][j] += ar[i] * bi[j] + ai[i] * br[j];
                }
        }
        const int64_t oC = (int64_t)b * sCb;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                int m = mt + i * MT, n = nt + j * NT;
                if (m < M && n < N) {
                    int64_t o = oC + m * sCm + n * sCn;
                    if (ACC) { Cr[o] += re[i][j]; Ci[o] += im[i][j]; }
                    else { Cr[o] = re[i][j]; Ci[o] = im[i][j]; }
                }
            }
    }
}

// tile shapes: R* for the p x p^2 per-box accumulators (one tile per
// thread), Z* for the mode products on p^2 x p and p x p operands
template <int P> struct Tiles;
template <> struct Tiles<18> { static constexpr int RM = 3, RN = 9, ZM = 3, ZN = 6; };
template <> struct Tiles<15> { static constexpr int RM = 3, RN = 5, ZM = 3, ZN = 5; };
template <> struct Tiles<9> { static constexpr int RM = 1, RN = 3, ZM = 3, ZN = 3; };

// store a p x p^2 register accumulator (tile layout of gemm_regs); COH: with
// relaxed agent-scope atomic stores (read by another workgroup of the same
// launch)
template <typename T, int P, bool COH = false, int RM, int RN>
__device__ inline void store_tiles(const T (&acc)[RM][RN], T *dst)
{
    constexpr int P2 = P * P, MT = (P + RM - 1) / RM, NT = (P2 + RN - 1) / RN;
    const int t = threadIdx.x;
    if (t >= MT * NT) return;
    const int mt = t / NT, nt = t % NT;
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            int m = mt + i * MT, n = nt + j * NT;
            if (m < P && n < P2) {
                if constexpr (COH)
                    __hip_atomic_store(dst + m * P2 + n, acc[i][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    dst[m * P2 + n] = acc[i][j];
            }
        }
}

// Lagrange basis of the Chebyshev nodes at xi (barycentric formula)
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

}  // namespace
}  // namespace dmk
