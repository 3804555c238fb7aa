// Step 0 of the discrete DMK algorithm (Sec. 3.5) on the GPU: root box,
// Morton keys, stable radix sort, the level-restricted adaptive tree (Sec.
// 3.3; octree in 3-D, quadtree in 2-D), colleagues, coarse neighbours, the
// flags F_leaf/F_out/F_in, per-level work lists and the residual interaction
// lists.
//
// Tree rules (each box refined into all 2^d children):
//  (1) a box holding more than n_s points is refined (below the depth cap);
//  (2) level restriction -- leaves sharing a boundary point differ by at most
//      one level -- holds iff every refined box Q at level l has all its
//      level-l neighbour regions present, i.e. their parents are refined.
// The set of refined boxes is the smallest set closed under (1) and (2).  It
// is computed by one sweep from the finest level upward: the refined boxes of
// level l force the parents of their 3^d neighbour regions at level l-1.
// Each box is identified by its Morton prefix; all lookups are binary
// searches in sorted prefix arrays, so the result does not depend on
// scheduling and is reproducible bit for bit.
//
// Several independent point sets (a batch of problems) form a forest: every
// key carries the problem index above its Morton bits, so a box key at level
// l is (problem << d l) | Morton prefix, level 0 holds one root per problem,
// and neighbour searches never leave a problem.  Each problem has its own
// root box from its own bounding box.

#include <algorithm>
#include <cmath>

#include "dmk_internal.h"
#include "prim.h"

namespace dmk {

namespace {

constexpr int TPB = 256;

template <int D> struct Geo;
template <> struct Geo<3> { static constexpr int NC = 8, NCOL = 27, NCO = 7, NRING = 64, KBMAX = 21; };
template <> struct Geo<2> { static constexpr int NC = 4, NCOL = 9, NCO = 3, NRING = 16, KBMAX = 31; };

__host__ __device__ inline uint64_t spread3(uint64_t v)
{
    // bit b of v -> bit 3b
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__host__ __device__ inline uint64_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return v;
}

__host__ __device__ inline uint64_t spread2(uint64_t v)
{
    // bit b of v -> bit 2b
    v &= 0xffffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

__host__ __device__ inline uint64_t compact2(uint64_t v)
{
    v &= 0x5555555555555555ull;
    v = (v ^ (v >> 1)) & 0x3333333333333333ull;
    v = (v ^ (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
    v = (v ^ (v >> 4)) & 0x00ff00ff00ff00ffull;
    v = (v ^ (v >> 8)) & 0x0000ffff0000ffffull;
    v = (v ^ (v >> 16)) & 0x00000000ffffffffull;
    return v;
}

// Morton interleave; x is the most significant coordinate inside each group
template <int D>
__host__ __device__ inline uint64_t morton(const int64_t *c)
{
    if (D == 3) return (spread3((uint64_t)c[0]) << 2) | (spread3((uint64_t)c[1]) << 1) | spread3((uint64_t)c[2]);
    return (spread2((uint64_t)c[0]) << 1) | spread2((uint64_t)c[1]);
}

// coordinates and problem of a box key at level l
template <int D>
__host__ __device__ inline void box_coords(uint64_t key, int l, int64_t *c)
{
    const uint64_t m = (l == 0) ? 0ull : (key & ((1ull << (D * l)) - 1ull));
    if (D == 3) {
        c[0] = (int64_t)compact3(m >> 2);
        c[1] = (int64_t)compact3(m >> 1);
        c[2] = (int64_t)compact3(m);
    } else {
        c[0] = (int64_t)compact2(m >> 1);
        c[1] = (int64_t)compact2(m);
    }
}

template <int D>
__host__ __device__ inline uint64_t box_pid(uint64_t key, int l)
{
    return key >> (D * l);
}

template <int D>
__host__ __device__ inline uint64_t box_key(uint64_t pid, int l, const int64_t *c)
{
    return (pid << (D * l)) | morton<D>(c);
}

// offset k of the 3^d neighbourhood, lexicographic (dx, dy[, dz]) from -1
template <int D>
__host__ __device__ inline void nbr_offset(int k, int64_t *d)
{
    if (D == 3) { d[0] = k / 9 - 1; d[1] = (k / 3) % 3 - 1; d[2] = k % 3 - 1; }
    else { d[0] = k / 3 - 1; d[1] = k % 3 - 1; }
}

__device__ inline int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int64_t find_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t i = lower_bound_u64(a, n, v);
    return (i < n && a[i] == v) ? i : -1;
}

// ---------------------------------------------------------------- kernels
template <int D>
__global__ void k_bbox_partial(const double *pts, int64_t n, double *part)
{
    __shared__ double red[7][TPB];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        for (int d = 0; d < D; ++d) {
            double v = pts[D * i + d];
            if (!isfinite(v)) bad = 1.0;
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    for (int d = 0; d < 3; ++d) { red[d][threadIdx.x] = mn[d]; red[3 + d][threadIdx.x] = mx[d]; }
    red[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
            }
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

// one block per problem: bounding box of its range [poff[b], poff[b+1])
template <int D>
__global__ void k_bbox_prob(const double *pts, const int64_t *poff, double *part)
{
    __shared__ double red[7][TPB];
    const int64_t b = blockIdx.x, i0 = poff[b], i1 = poff[b + 1];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double bad = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += TPB)
        for (int d = 0; d < D; ++d) {
            double v = pts[D * i + d];
            if (!isfinite(v)) bad = 1.0;
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    for (int d = 0; d < 3; ++d) { red[d][threadIdx.x] = mn[d]; red[3 + d][threadIdx.x] = mx[d]; }
    red[6][threadIdx.x] = bad;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
            }
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[b * 7 + threadIdx.x] = red[threadIdx.x][0];
}

// point keys: problem index (binary search in poff) above the Morton bits of
// floor((x' + 1/2) 2^kb) per axis, x' = (x - centre_b)/side_b
#pragma clang fp contract(off)
template <int D>
__global__ void k_keys(const double *pts, int64_t n, const int64_t *poff, int nprob, const double *pcenter,
                       const double *pside, int kb, double *xn, uint64_t *keys, int32_t *idx)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nprob;  // last b with poff[b] <= i
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (poff[mid] <= i) lo = mid; else hi = mid;
    }
    const int b = lo;
    const double scale = ldexp(1.0, kb);
    const double side = pside[b];
    int64_t k[3];
    for (int d = 0; d < D; ++d) {
        double x = (pts[D * i + d] - pcenter[D * b + d]) / side;
        xn[d * n + i] = x;
        double f = floor((x + 0.5) * scale);
        uint64_t kk = (f <= 0.0) ? 0ull : (uint64_t)f;
        if (kk > (1ull << kb) - 1ull) kk = (1ull << kb) - 1ull;
        k[d] = (int64_t)kk;
    }
    keys[i] = box_key<D>((uint64_t)b, kb, k);
    idx[i] = (int32_t)i;
}
#pragma clang fp contract(on)

template <int D>
__global__ void k_gather_points(const double *xn, const int32_t *perm, int64_t n, double *X, double *Y,
                                double *Z)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    X[i] = xn[j];
    Y[i] = xn[n + j];
    if (D == 3) Z[i] = xn[2 * n + j];
}

// children of the refined prefixes of one level
template <int D>
__global__ void k_children(const uint64_t *ref, int64_t m, uint64_t *out)
{
    constexpr int NC = Geo<D>::NC;
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= NC * m) return;
    out[i] = (ref[i / NC] << D) | (uint64_t)(i % NC);
}

template <int D>
__device__ inline void prefix_range(const uint64_t *keys, int64_t n, uint64_t P, int l, int kb, int64_t *lo,
                                    int64_t *hi)
{
    int sh = D * (kb - l);
    *lo = lower_bound_u64(keys, n, P << sh);
    *hi = lower_bound_u64(keys, n, (P + 1) << sh);
}

template <int D>
__global__ void k_refine_flag(const uint64_t *ex, int64_t m, int l, int kb, const uint64_t *keys, int64_t n,
                              int ns, uint8_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= m) return;
    int64_t a, b;
    prefix_range<D>(keys, n, ex[i], l, kb, &a, &b);
    flag[i] = (b - a > ns) ? 1 : 0;
}

// parents (level l-1) of the 3^d level-l neighbour regions of each refined box
template <int D>
__global__ void k_balance_cands(const uint64_t *ref, int64_t m, int l, uint64_t *out)
{
    constexpr int NCOL = Geo<D>::NCOL;
    int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (t >= NCOL * m) return;
    int64_t i = t / NCOL;
    int k = (int)(t % NCOL);
    int64_t c[3], d[3], q[3];
    box_coords<D>(ref[i], l, c);
    const uint64_t pid = box_pid<D>(ref[i], l);
    nbr_offset<D>(k, d);
    int64_t lim = (int64_t)1 << l;
    uint64_t res = ~0ull;
    bool ok = true;
    for (int a = 0; a < D; ++a) {
        q[a] = c[a] + d[a];
        if (q[a] < 0 || q[a] >= lim) ok = false;
        q[a] >>= 1;
    }
    if (ok) res = box_key<D>(pid, l - 1, q);
    out[t] = res;
}

template <int D>
__global__ void k_box_fill(int l, int kb, int64_t b0, int64_t nb, const uint64_t *bkey_all, int64_t prev0,
                           int64_t nprev, int64_t next0, const uint64_t *ref, int64_t nref,
                           const uint64_t *keys, int64_t n, int ns, int32_t *blevel, int32_t *parent,
                           int32_t *child0, int32_t *pstart, int32_t *pcount, uint8_t *bflags,
                           double *bcenter, int32_t *bprob)
{
    constexpr int NC = Geo<D>::NC;
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    uint64_t P = bkey_all[b];
    blevel[b] = l;
    int64_t a, e;
    prefix_range<D>(keys, n, P, l, kb, &a, &e);
    pstart[b] = (int32_t)a;
    pcount[b] = (int32_t)(e - a);
    int64_t r = (nref > 0) ? find_u64(ref, nref, P) : -1;
    bool leaf = r < 0;
    child0[b] = leaf ? -1 : (int32_t)(next0 + NC * r);
    parent[b] = (l == 0) ? -1 : (int32_t)(prev0 + find_u64(bkey_all + prev0, nprev, P >> D));
    uint8_t f = leaf ? 1 : 0;
    if (!leaf && (e - a) > ns) f |= 2;
    bflags[b] = f;
    bprob[b] = (int32_t)box_pid<D>(P, l);
    int64_t c[3];
    box_coords<D>(P, l, c);
    double s = ldexp(1.0, -l);
    for (int d = 0; d < D; ++d) bcenter[D * b + d] = -0.5 + ((double)c[d] + 0.5) * s;
}

template <int D>
__global__ void k_colleagues(int l, int64_t b0, int64_t nb, const uint64_t *bkey_all, int32_t *col)
{
    constexpr int NCOL = Geo<D>::NCOL;
    int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (t >= NCOL * nb) return;
    int64_t i = t / NCOL;
    int k = (int)(t % NCOL);
    const uint64_t K = bkey_all[b0 + i];
    int64_t c[3], d[3], q[3];
    box_coords<D>(K, l, c);
    nbr_offset<D>(k, d);
    int64_t lim = (int64_t)1 << l;
    int32_t res = -1;
    bool ok = true;
    for (int a = 0; a < D; ++a) {
        q[a] = c[a] + d[a];
        if (q[a] < 0 || q[a] >= lim) ok = false;
    }
    if (ok) {
        int64_t f = find_u64(bkey_all + b0, nb, box_key<D>(box_pid<D>(K, l), l, q));
        if (f >= 0) res = (int32_t)(b0 + f);
    }
    col[(b0 + i) * NCOL + k] = res;
}

template <int D>
__global__ void k_flags2(int64_t nbox, const int32_t *col, const int32_t *parent, uint8_t *bflags)
{
    constexpr int NCOL = Geo<D>::NCOL;
    int64_t b = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (b >= nbox) return;
    uint8_t f = bflags[b];
    bool fin = false;
    for (int k = 0; k < NCOL; ++k) {
        int32_t j = col[b * NCOL + k];
        if (j >= 0 && (bflags[j] & 2)) fin = true;
    }
    bool fout = f & 2;
    int32_t par = parent[b];
    bool term = !fout && (par < 0 || (bflags[par] & 2));
    f |= (fin ? 4 : 0) | (term ? 8 : 0);
    bflags[b] = f;  // bits 0-1 are only read by other threads, bits 2-3 only written here
}

template <int D>
__global__ void k_coarse(int l, int64_t b0, int64_t nb, const uint64_t *bkey_all, int64_t prev0,
                         int64_t nprev, const uint8_t *bflags, int32_t *ncoarse, int32_t *coarse)
{
    constexpr int NCOL = Geo<D>::NCOL, NCO = Geo<D>::NCO;
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    int cnt = 0;
    int32_t found[NCO];
    if (l > 0 && (bflags[b] & 1)) {
        uint64_t P = bkey_all[b];
        int64_t c[3], d[3], q[3];
        box_coords<D>(P, l, c);
        const uint64_t pid = box_pid<D>(P, l);
        int64_t lim = (int64_t)1 << l;
        for (int k = 0; k < NCOL; ++k) {
            nbr_offset<D>(k, d);
            bool ok = true;
            for (int a = 0; a < D; ++a) {
                q[a] = c[a] + d[a];
                if (q[a] < 0 || q[a] >= lim) ok = false;
                q[a] >>= 1;
            }
            if (!ok) continue;
            uint64_t Q = box_key<D>(pid, l - 1, q);
            if (Q == (P >> D)) continue;
            int64_t f = find_u64(bkey_all + prev0, nprev, Q);
            if (f < 0) continue;
            int32_t j = (int32_t)(prev0 + f);
            if (!(bflags[j] & 1)) continue;
            bool dup = false;
            for (int m = 0; m < cnt; ++m) dup |= (found[m] == j);
            if (!dup && cnt < NCO) found[cnt++] = j;
        }
    }
    ncoarse[b] = cnt;
    for (int m = 0; m < NCO; ++m) coarse[b * NCO + m] = (m < cnt) ? found[m] : -1;
}

// ------------------------------------------------------------ small helpers
template <typename T>
T *talloc(Plan *P, int64_t count)
{
    return (T *)dalloc(P, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

struct Scratch {  // temporary device buffers freed at the end of the plan build
    std::vector<void *> ptrs;
    template <typename T>
    T *get(int64_t count)
    {
        void *p = nullptr;
        DMK_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
        ptrs.push_back(p);
        return (T *)p;
    }
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

// sorted unique union of uint64 arrays (removes the ~0 sentinel)
int64_t sort_unique(Scratch &S, uint64_t *in, int64_t n, uint64_t **out, hipStream_t s)
{
    if (n == 0) { *out = S.get<uint64_t>(1); return 0; }
    uint64_t *sorted = S.get<uint64_t>(n);
    prim::sort_pairs(S, (const uint64_t *)in, sorted, (const int32_t *)nullptr, (int32_t *)nullptr, n, 64, s);
    uint64_t *uniq = S.get<uint64_t>(n);
    int64_t *cnt = S.get<int64_t>(1);
    prim::unique_sorted(S, (const uint64_t *)sorted, uniq, cnt, n, s);
    int64_t m = 0;
    DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DMK_HIP(hipStreamSynchronize(s));
    if (m > 0) {
        uint64_t last = 0;
        DMK_HIP(hipMemcpy(&last, uniq + m - 1, sizeof(uint64_t), hipMemcpyDeviceToHost));
        if (last == ~0ull) m--;
    }
    *out = uniq;
    return m;
}

}  // namespace

template <int D>
static void build_tree_t(Plan *P, const double *pts, hipStream_t s)
{
    constexpr int NC = Geo<D>::NC, NCOL = Geo<D>::NCOL, NCO = Geo<D>::NCO;
    const int64_t n = P->n;
    const int nprob = P->nprob;
    const int kb = P->kb;
    Scratch S;
    // ---- root box of each problem from its bounding box
    std::vector<double> bbx(7 * (size_t)nprob, 0.0);
    if (n > 0 && !P->fixed_root) {
        if (nprob == 1) {
            int nb = (int)std::min<int64_t>(1024, (n + TPB - 1) / TPB);
            double *part = S.get<double>(7 * nb);
            hipLaunchKernelGGL(k_bbox_partial<D>, dim3(nb), dim3(TPB), 0, s, pts, n, part);
            std::vector<double> h(7 * nb);
            DMK_HIP(hipMemcpyAsync(h.data(), part, 7 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
            for (int k = 0; k < 7; ++k) bbx[k] = h[k];
            for (int b = 0; b < nb; ++b) {
                for (int d = 0; d < 3; ++d) {
                    bbx[d] = std::min(bbx[d], h[7 * b + d]);
                    bbx[3 + d] = std::max(bbx[3 + d], h[7 * b + 3 + d]);
                }
                bbx[6] = std::max(bbx[6], h[7 * b + 6]);
            }
        } else {
            double *part = S.get<double>(7 * (int64_t)nprob);
            hipLaunchKernelGGL(k_bbox_prob<D>, dim3(nprob), dim3(TPB), 0, s, pts, P->d_poff, part);
            DMK_HIP(hipMemcpyAsync(bbx.data(), part, 7 * (size_t)nprob * sizeof(double), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
        }
        for (int b = 0; b < nprob; ++b)
            if (bbx[7 * b + 6] != 0.0) throw Error{DMK_ERR_ARG, "non-finite point coordinate"};
    }
    P->pcenter.assign((size_t)nprob * D, 0.0);
    P->pside.assign(nprob, 1.0);
    for (int b = 0; b < nprob; ++b) {
        double ext = 0.0;
        const bool empty = P->poff[b + 1] == P->poff[b];
        for (int d = 0; d < D; ++d) {
            double lo = bbx[7 * b + d], hi = bbx[7 * b + 3 + d];
            if (empty) lo = hi = 0.0;
            P->pcenter[(size_t)D * b + d] = 0.5 * (lo + hi);
            if (hi - lo > ext) ext = hi - lo;
        }
        P->pside[b] = (ext > 0.0) ? ext * (1.0 + std::ldexp(1.0, -40)) : 1.0;
    }
    if (P->fixed_root) {  // the unit cube centred at the origin (volume plans: nprob = 1)
        for (int d = 0; d < D; ++d) P->pcenter[d] = 0.0;
        P->pside[0] = 1.0;
    }
    for (int d = 0; d < D; ++d) P->center[d] = P->pcenter[d];
    P->side = P->pside[0];
    P->d_pcenter = talloc<double>(P, (int64_t)nprob * D);
    P->d_pside = talloc<double>(P, nprob);
    DMK_HIP(hipMemcpyAsync(P->d_pcenter, P->pcenter.data(), (size_t)nprob * D * sizeof(double),
                           hipMemcpyHostToDevice, s));
    DMK_HIP(hipMemcpyAsync(P->d_pside, P->pside.data(), (size_t)nprob * sizeof(double), hipMemcpyHostToDevice, s));

    // ---- keys, sort, sorted coordinates
    P->X = talloc<double>(P, n);
    P->Y = talloc<double>(P, n);
    P->Z = (D == 3) ? talloc<double>(P, n) : nullptr;
    P->perm = talloc<int32_t>(P, n);
    P->keys = talloc<uint64_t>(P, n);
    if (n > 0) {
        double *xn = S.get<double>(D * n);
        uint64_t *k0 = S.get<uint64_t>(n);
        int32_t *i0 = S.get<int32_t>(n);
        hipLaunchKernelGGL(k_keys<D>, dim3(nblk(n)), dim3(TPB), 0, s, pts, n, P->d_poff, nprob, P->d_pcenter,
                           P->d_pside, kb, xn, k0, i0);
        const int endbit = D * kb + P->pbits;
        prim::sort_pairs(S, (const uint64_t *)k0, P->keys, (const int32_t *)i0, P->perm, n, endbit, s);
        hipLaunchKernelGGL(k_gather_points<D>, dim3(nblk(n)), dim3(TPB), 0, s, xn, P->perm, n, P->X, P->Y, P->Z);
    }

    // ---- refinement by count (level 0: one root per problem)
    const int maxd = P->max_depth;
    std::vector<uint64_t *> ref(maxd + 2, nullptr);
    std::vector<int64_t> nref(maxd + 2, 0);
    uint64_t *ex = S.get<uint64_t>(nprob);
    {
        std::vector<uint64_t> roots(nprob);
        for (int b = 0; b < nprob; ++b) roots[b] = (uint64_t)b;
        DMK_HIP(hipMemcpyAsync(ex, roots.data(), nprob * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        DMK_HIP(hipStreamSynchronize(s));
    }
    int64_t nex = nprob;
    for (int l = 0; l < maxd && n > 0; ++l) {
        if (l > 0) {
            nex = NC * nref[l - 1];
            ex = S.get<uint64_t>(nex);
            hipLaunchKernelGGL(k_children<D>, dim3(nblk(nex)), dim3(TPB), 0, s, ref[l - 1], nref[l - 1], ex);
        }
        uint8_t *flag = S.get<uint8_t>(nex);
        hipLaunchKernelGGL(k_refine_flag<D>, dim3(nblk(nex)), dim3(TPB), 0, s, ex, nex, l, kb, P->keys, n,
                           P->leaf_max, flag);
        uint64_t *sel = S.get<uint64_t>(nex);
        int64_t *cnt = S.get<int64_t>(1);
        prim::select_flagged(S, (const uint64_t *)ex, (uint64_t)0, (const uint8_t *)flag, sel, cnt, nex, s);
        int64_t m = 0;
        DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        ref[l] = sel;
        nref[l] = m;
        if (m == 0) break;
    }
    // ---- level restriction: finest refined level upward
    int lmax = -1;
    for (int l = 0; l < maxd; ++l)
        if (nref[l] > 0) lmax = l;
    for (int l = lmax; l >= 1; --l) {
        if (nref[l] == 0) continue;
        int64_t nc = NCOL * nref[l];
        uint64_t *cand = S.get<uint64_t>(nc + nref[l - 1]);
        hipLaunchKernelGGL(k_balance_cands<D>, dim3(nblk(nc)), dim3(TPB), 0, s, ref[l], nref[l], l, cand);
        if (nref[l - 1] > 0)
            DMK_HIP(hipMemcpyAsync(cand + nc, ref[l - 1], nref[l - 1] * sizeof(uint64_t),
                                   hipMemcpyDeviceToDevice, s));
        uint64_t *merged = nullptr;
        int64_t m = sort_unique(S, cand, nc + nref[l - 1], &merged, s);
        ref[l - 1] = merged;
        nref[l - 1] = m;
    }

    // ---- materialise boxes level by level
    std::vector<int64_t> lstart(1, 0);
    std::vector<int64_t> cnts;
    cnts.push_back(nprob);
    for (int l = 1; l <= maxd; ++l) {
        if (nref[l - 1] == 0) break;
        cnts.push_back(NC * nref[l - 1]);
    }
    P->nlevels = (int)cnts.size();
    for (int64_t c : cnts) lstart.push_back(lstart.back() + c);
    P->level_start = lstart;
    const int64_t nbox = lstart.back();
    P->nbox = nbox;
    P->bkey = talloc<uint64_t>(P, nbox);
    P->blevel = talloc<int32_t>(P, nbox);
    P->parent = talloc<int32_t>(P, nbox);
    P->child0 = talloc<int32_t>(P, nbox);
    P->pstart = talloc<int32_t>(P, nbox);
    P->pcount = talloc<int32_t>(P, nbox);
    P->bflags = talloc<uint8_t>(P, nbox);
    P->bprob = talloc<int32_t>(P, nbox);
    P->colleague = talloc<int32_t>(P, NCOL * nbox);
    P->ncoarse = talloc<int32_t>(P, nbox);
    P->coarse = talloc<int32_t>(P, NCO * nbox);
    P->bcenter = talloc<double>(P, D * nbox);
    {
        std::vector<uint64_t> roots(nprob);
        for (int b = 0; b < nprob; ++b) roots[b] = (uint64_t)b;
        DMK_HIP(hipMemcpyAsync(P->bkey, roots.data(), nprob * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        DMK_HIP(hipStreamSynchronize(s));
    }
    for (int l = 1; l < P->nlevels; ++l)
        hipLaunchKernelGGL(k_children<D>, dim3(nblk(cnts[l])), dim3(TPB), 0, s, ref[l - 1], nref[l - 1],
                           P->bkey + lstart[l]);
    for (int l = 0; l < P->nlevels; ++l) {
        int64_t prev0 = (l > 0) ? lstart[l - 1] : 0, nprev = (l > 0) ? cnts[l - 1] : 0;
        int64_t next0 = lstart[l + 1];
        hipLaunchKernelGGL(k_box_fill<D>, dim3(nblk(cnts[l])), dim3(TPB), 0, s, l, kb, lstart[l], cnts[l], P->bkey,
                           prev0, nprev, next0, ref[l], (l < maxd) ? nref[l] : (int64_t)0, P->keys, n,
                           P->leaf_max, P->blevel, P->parent, P->child0, P->pstart, P->pcount, P->bflags,
                           P->bcenter, P->bprob);
    }
    for (int l = 0; l < P->nlevels; ++l)
        hipLaunchKernelGGL(k_colleagues<D>, dim3(nblk(NCOL * cnts[l])), dim3(TPB), 0, s, l, lstart[l], cnts[l],
                           P->bkey, P->colleague);
    hipLaunchKernelGGL(k_flags2<D>, dim3(nblk(nbox)), dim3(TPB), 0, s, nbox, P->colleague, P->parent, P->bflags);
    for (int l = 0; l < P->nlevels; ++l) {
        int64_t prev0 = (l > 0) ? lstart[l - 1] : 0, nprev = (l > 0) ? cnts[l - 1] : 0;
        hipLaunchKernelGGL(k_coarse<D>, dim3(nblk(cnts[l])), dim3(TPB), 0, s, l, lstart[l], cnts[l], P->bkey,
                           prev0, nprev, P->bflags, P->ncoarse, P->coarse);
    }
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

void build_tree(Plan *P, const double *pts, hipStream_t s)
{
    if (P->dim == 3) build_tree_t<3>(P, pts, s);
    else build_tree_t<2>(P, pts, s);
    // sources and targets are the union's points until split_roles
    P->nsrc = P->ntgt = P->n;
    P->Xs = P->Xt = P->X;
    P->Ys = P->Yt = P->Y;
    P->Zs = P->Zt = P->Z;
    P->sperm = P->tperm = P->perm;
    P->sstart = P->tstart = P->pstart;
    P->scount = P->tcount = P->pcount;
}

namespace {

// role flags of the union's points in tree order: 1 for a source
__global__ void k_role_flags(const int32_t *perm, int64_t n, int64_t nsrc, int32_t *fs, int32_t *ft)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i > n) return;
    const int32_t src = (i < n && perm[i] < nsrc) ? 1 : 0;
    fs[i] = (i < n) ? src : 0;  // a trailing zero: the exclusive scan's entry n is the total
    ft[i] = (i < n) ? 1 - src : 0;
}

__global__ void k_role_scatter(const double *X, const double *Y, const double *Z, const int32_t *perm, int64_t n,
                               int64_t nsrc, const int32_t *fs, const int32_t *sr, const int32_t *tr, double *Xs,
                               double *Ys, double *Zs, int32_t *sperm, double *Xt, double *Yt, double *Zt,
                               int32_t *tperm)
{
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    if (fs[i]) {
        const int32_t k = sr[i];
        Xs[k] = X[i];
        Ys[k] = Y[i];
        if (Z) Zs[k] = Z[i];
        sperm[k] = perm[i];
    } else {
        const int32_t k = tr[i];
        Xt[k] = X[i];
        Yt[k] = Y[i];
        if (Z) Zt[k] = Z[i];
        tperm[k] = (int32_t)(perm[i] - nsrc);
    }
}

// per box: its sources and its targets, from the ranks at its union range
__global__ void k_role_ranges(const int32_t *pstart, const int32_t *pcount, int64_t nbox, const int32_t *sr,
                              const int32_t *tr, int32_t *sstart, int32_t *scount, int32_t *tstart, int32_t *tcount)
{
    const int64_t b = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (b >= nbox) return;
    const int32_t a = pstart[b], e = pstart[b] + pcount[b];
    sstart[b] = sr[a];
    scount[b] = sr[e] - sr[a];
    tstart[b] = tr[a];
    tcount[b] = tr[e] - tr[a];
}

}  // namespace

void split_roles(Plan *P, hipStream_t s)
{
    Scratch S;
    const int64_t n = P->n, nbox = P->nbox, ns = P->nsrc, nt = n - ns;
    int32_t *fs = S.get<int32_t>(n + 1), *ft = S.get<int32_t>(n + 1);
    int32_t *sr = S.get<int32_t>(n + 1), *tr = S.get<int32_t>(n + 1);
    hipLaunchKernelGGL(k_role_flags, dim3(nblk(n + 1)), dim3(TPB), 0, s, P->perm, n, ns, fs, ft);
    prim::exclusive_scan(S, fs, sr, n + 1, s);
    prim::exclusive_scan(S, ft, tr, n + 1, s);
    const bool d3 = P->dim == 3;
    P->Xs = talloc<double>(P, ns);
    P->Ys = talloc<double>(P, ns);
    P->Zs = d3 ? talloc<double>(P, ns) : nullptr;
    P->sperm = talloc<int32_t>(P, ns);
    P->Xt = talloc<double>(P, nt);
    P->Yt = talloc<double>(P, nt);
    P->Zt = d3 ? talloc<double>(P, nt) : nullptr;
    P->tperm = talloc<int32_t>(P, nt);
    P->sstart = talloc<int32_t>(P, nbox);
    P->scount = talloc<int32_t>(P, nbox);
    P->tstart = talloc<int32_t>(P, nbox);
    P->tcount = talloc<int32_t>(P, nbox);
    if (n > 0)
        hipLaunchKernelGGL(k_role_scatter, dim3(nblk(n)), dim3(TPB), 0, s, P->X, P->Y, P->Z, P->perm, n, ns,
                           (const int32_t *)fs, (const int32_t *)sr, (const int32_t *)tr, P->Xs, P->Ys, P->Zs,
                           P->sperm, P->Xt, P->Yt, P->Zt, P->tperm);
    hipLaunchKernelGGL(k_role_ranges, dim3(nblk(nbox)), dim3(TPB), 0, s, P->pstart, P->pcount, nbox,
                       (const int32_t *)sr, (const int32_t *)tr, P->sstart, P->scount, P->tstart, P->tcount);
    P->ntgt = nt;
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ lists
namespace {

__global__ void k_list_flags(int64_t nbox, const uint8_t *bflags, const int32_t *pcount, uint8_t *f_fout,
                             uint8_t *f_fin, uint8_t *f_leaf)
{
    int64_t b = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (b >= nbox) return;
    uint8_t f = bflags[b];
    bool ne = pcount[b] > 0;
    f_fout[b] = (f & 2) ? 1 : 0;
    f_fin[b] = (ne && (f & 4)) ? 1 : 0;
    f_leaf[b] = (ne && (f & 1)) ? 1 : 0;
}

// targets grouped by anchor: per leaf, its anchor's slot, and per anchor the
// number of targets
__global__ void k_leaf_keys(const int32_t *leaves, int64_t nleaf, const int32_t *anchor, const int32_t *local_slot,
                            const int32_t *pcount, int32_t *key, int32_t *ident, int32_t *anc_cnt)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nleaf) return;
    int32_t L = leaves[i];
    int32_t a = local_slot[anchor[L]];
    key[i] = a;
    ident[i] = L;
    atomicAdd(&anc_cnt[a], pcount[L]);
}

__global__ void k_leaf_counts(const int32_t *sorted_leaves, int64_t nleaf, const int32_t *pcount, int32_t *cnt)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < nleaf) cnt[i] = pcount[sorted_leaves[i]];
}

__global__ void k_fill_targets(const int32_t *sorted_leaves, int64_t nleaf, const int32_t *pstart,
                               const int32_t *pcount, const int32_t *pos, int32_t *tgt)
{
    int64_t i = blockIdx.x;
    if (i >= nleaf) return;
    int32_t L = sorted_leaves[i];
    for (int k = threadIdx.x; k < pcount[L]; k += TPB) tgt[pos[i] + k] = pstart[L] + k;
}

// anchors whose local values a finer anchor reads (its parent's anchor)
__global__ void k_anchor_read(const int32_t *anc, int64_t m, const int32_t *blevel, const int32_t *parent,
                              const int32_t *anchor, const int32_t *local_slot, uint8_t *read)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= m) return;
    const int32_t B = anc[i];
    if (blevel[B] > 0) read[local_slot[anchor[parent[B]]]] = 1;
}

__global__ void k_slots(const int32_t *list, int64_t m, int32_t *slot)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < m) slot[list[i]] = (int32_t)i;
}

__global__ void k_nonempty(const int32_t *pcount, int64_t m, uint8_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < m) flag[i] = pcount[i] > 0 ? 1 : 0;
}

// parents of the non-empty F_in boxes of levels >= 1
__global__ void k_oct_flag(const int32_t *fin, int64_t m, const int32_t *parent, uint8_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= m) return;
    int32_t P = parent[fin[i]];
    if (P >= 0) flag[P] = 1;
}

// sibling group of parent P: child k (bits x y [z]) sits at cell k + (1,..,1)
// of the 4^d block; cell g holds child ((g+1) & 1) of P's colleague at
// offset (g+1)/2 - 1 per axis
template <int D>
__global__ void k_oct_fill(const int32_t *octs, int64_t m, const int32_t *child0, const int32_t *col,
                           const uint8_t *bflags, const int32_t *blevel, const int32_t *bprob,
                           const int32_t *proxy_slot, const int32_t *psi_slot, int32_t *dst, int32_t *src,
                           int32_t *lev, int32_t *prob)
{
    constexpr int NC = Geo<D>::NC, NCOL = Geo<D>::NCOL, NR = Geo<D>::NRING;
    int64_t i = blockIdx.x;
    if (i >= m) return;
    const int32_t P = octs[i];
    const int t = threadIdx.x;
    if (t < NC) dst[i * NC + t] = psi_slot[child0[P] + t];
    if (t == 0) {
        lev[i] = blevel[P] + 1;
        prob[i] = bprob[P];
    }
    if (t < NR) {
        int k = 0, c = 0, r = t;
        int g[3];
        for (int a = D - 1; a >= 0; --a) { g[a] = r % 4; r /= 4; }
        for (int a = 0; a < D; ++a) {
            k = 3 * k + (g[a] + 1) / 2;      // colleague offset + 1
            c = 2 * c + ((g[a] + 1) & 1);   // child bit
        }
        int32_t C = col[(int64_t)P * NCOL + k];
        int32_t v = -1;
        if (C >= 0 && child0[C] >= 0) {
            int32_t S = child0[C] + c;
            if (bflags[S] & 2) v = proxy_slot[S];
        }
        src[i * NR + t] = v;
    }
}

// anchor of a box: itself if it holds points and has F_in, else its parent's
// anchor; the root is always an anchor.  One launch per level, top down.
__global__ void k_anchor(int64_t b0, int64_t nb, const int32_t *parent, const uint8_t *f_fin, int32_t *anchor)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nb) return;
    int64_t b = b0 + i;
    anchor[b] = (parent[b] < 0 || f_fin[b]) ? (int32_t)b : anchor[parent[b]];
}

// residual lists, gather form: for target leaf B, the terminal non-empty
// boxes among (a) the colleagues of B and of each of its ancestors and
// (b) the leaves one level finer that share a boundary point with B.
template <int D, bool FILL>
__global__ void k_near_lists(const int32_t *leaves, int64_t nleaf, const int32_t *lstart_dev, int nlevels,
                             const uint64_t *bkey, const int32_t *blevel, const int32_t *parent,
                             const int32_t *col, const uint8_t *bflags, const int32_t *pcount,
                             const int32_t *tcount, int32_t *count, const int32_t *off, int32_t *src, int32_t *pre,
                             int64_t *pairs)
{
    constexpr int NCOL = Geo<D>::NCOL, NR = Geo<D>::NRING;
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= nleaf) return;
    int32_t B = leaves[i];
    int cnt = 0;
    int64_t pr = 0;
    int32_t base = FILL ? off[i] : 0;
    // pre: running count of source points before each entry (FILL pass)
    for (int32_t A = B; A >= 0; A = parent[A])
        for (int k = 0; k < NCOL; ++k) {
            int32_t T = col[(int64_t)A * NCOL + k];
            if (T >= 0 && (bflags[T] & 8) && pcount[T] > 0) {
                if (FILL) { src[base + cnt] = T; pre[base + i + cnt] = (int32_t)pr; }
                cnt++;
                pr += pcount[T];
            }
        }
    int l = blevel[B];
    if (l + 1 < nlevels) {
        int64_t c[3];
        box_coords<D>(bkey[B], l, c);
        const uint64_t pid = box_pid<D>(bkey[B], l);
        int64_t lim = (int64_t)1 << (l + 1);
        int64_t n1 = lstart_dev[l + 2] - lstart_dev[l + 1];
        const uint64_t *k1 = bkey + lstart_dev[l + 1];
        for (int r = 0; r < NR; ++r) {
            int64_t o[3], q[3];
            int rr = r;
            for (int a = D - 1; a >= 0; --a) { o[a] = rr % 4 - 1; rr /= 4; }
            bool own = true, ok = true;
            for (int a = 0; a < D; ++a) {
                if (o[a] < 0 || o[a] > 1) own = false;
                q[a] = 2 * c[a] + o[a];
                if (q[a] < 0 || q[a] >= lim) ok = false;
            }
            if (own || !ok) continue;
            int64_t f = find_u64(k1, n1, box_key<D>(pid, l + 1, q));
            if (f < 0) continue;
            int32_t T = (int32_t)(lstart_dev[l + 1] + f);
            if ((bflags[T] & 1) && (bflags[T] & 8) && pcount[T] > 0) {
                if (FILL) { src[base + cnt] = T; pre[base + i + cnt] = (int32_t)pr; }
                cnt++;
                pr += pcount[T];
            }
        }
    }
    if (FILL) pre[base + i + cnt] = (int32_t)pr;  // total after the last entry (one extra slot per leaf)
    if (!FILL) {
        count[i] = cnt;
        pairs[i] = pr * tcount[B];
    }
}

int64_t select_indices(Scratch &S, const uint8_t *flag, int64_t first, int64_t count, int32_t *out,
                       hipStream_t s)
{
    if (count == 0) return 0;
    int64_t *cnt = S.get<int64_t>(1);
    prim::select_flagged(S, (const int32_t *)nullptr, (int32_t)first, flag + first, out, cnt, count, s);
    int64_t m = 0;
    DMK_HIP(hipMemcpyAsync(&m, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DMK_HIP(hipStreamSynchronize(s));
    return m;
}

}  // namespace

template <int D>
static void build_lists_t(Plan *P, hipStream_t s)
{
    constexpr int NC = Geo<D>::NC, NR = Geo<D>::NRING;
    Scratch S;
    const int64_t nbox = P->nbox;
    const int L = P->nlevels;
    uint8_t *f_fout = S.get<uint8_t>(nbox), *f_fin = S.get<uint8_t>(nbox), *f_leaf = S.get<uint8_t>(nbox);
    // boxes that need local values and leaves to evaluate: those holding targets
    hipLaunchKernelGGL(k_list_flags, dim3(nblk(nbox)), dim3(TPB), 0, s, nbox, P->bflags, P->tcount, f_fout, f_fin,
                       f_leaf);
    P->l_fout = talloc<int32_t>(P, nbox);
    P->l_fin = talloc<int32_t>(P, nbox);
    P->l_anc = talloc<int32_t>(P, nbox + P->nprob);
    P->l_leaf = talloc<int32_t>(P, nbox);
    P->anchor = talloc<int32_t>(P, nbox);
    auto &ll = P->ll;
    ll.fout_off.assign(L + 1, 0);
    ll.fin_off.assign(L + 1, 0);
    ll.anc_off.assign(L + 1, 0);
    ll.leaf_off.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) {
        int64_t b0 = P->level_start[l], nb = P->level_start[l + 1] - b0;
        ll.fout_off[l + 1] = ll.fout_off[l] + select_indices(S, f_fout, b0, nb, P->l_fout + ll.fout_off[l], s);
        ll.fin_off[l + 1] = ll.fin_off[l] + select_indices(S, f_fin, b0, nb, P->l_fin + ll.fin_off[l], s);
        ll.leaf_off[l + 1] = ll.leaf_off[l] + select_indices(S, f_leaf, b0, nb, P->l_leaf + ll.leaf_off[l], s);
        hipLaunchKernelGGL(k_anchor, dim3(nblk(nb)), dim3(TPB), 0, s, b0, nb, P->parent, f_fin, P->anchor);
    }
    // anchors: the roots holding points, then the non-empty F_in boxes of
    // levels >= 1
    {
        uint8_t *f_root = S.get<uint8_t>(P->nprob);
        hipLaunchKernelGGL(k_nonempty, dim3(nblk(P->nprob)), dim3(TPB), 0, s, P->tcount, (int64_t)P->nprob, f_root);
        ll.anc_off[0] = 0;
        ll.anc_off[1] = select_indices(S, f_root, 0, P->nprob, P->l_anc, s);
        for (int l = 1; l < L; ++l) {
            int64_t m = ll.fin_off[l + 1] - ll.fin_off[l];
            if (m)
                DMK_HIP(hipMemcpyAsync(P->l_anc + ll.anc_off[l], P->l_fin + ll.fin_off[l], m * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, s));
            ll.anc_off[l + 1] = ll.anc_off[l] + m;
        }
    }
    P->nfout = ll.fout_off[L];
    P->nfin = ll.fin_off[L];
    P->nanc = ll.anc_off[L];
    P->nleaf = ll.leaf_off[L];
    P->max_fin_level = 0;
    P->max_fout_level = 0;
    for (int l = 0; l < L; ++l) {
        P->max_fin_level = std::max(P->max_fin_level, ll.fin_off[l + 1] - ll.fin_off[l]);
        P->max_fout_level = std::max(P->max_fout_level, ll.fout_off[l + 1] - ll.fout_off[l]);
    }
    // the upward pass's queue: the F_out boxes finest level first
    P->l_fout_up = talloc<int32_t>(P, std::max<int64_t>(P->nfout, 1));
    for (int l = L - 1, pos = 0; l >= 0; --l) {
        const int64_t m = ll.fout_off[l + 1] - ll.fout_off[l];
        if (m)
            DMK_HIP(hipMemcpyAsync(P->l_fout_up + pos, P->l_fout + ll.fout_off[l], m * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
        pos += (int)m;
    }
    P->q_fail = talloc<int32_t>(P, 1);
    DMK_HIP(hipMemsetAsync(P->q_fail, 0, sizeof(int32_t), s));
    P->proxy_slot = talloc<int32_t>(P, nbox);
    P->local_slot = talloc<int32_t>(P, nbox);
    P->psi_slot = talloc<int32_t>(P, nbox);
    DMK_HIP(hipMemsetAsync(P->proxy_slot, 0xff, nbox * sizeof(int32_t), s));
    DMK_HIP(hipMemsetAsync(P->local_slot, 0xff, nbox * sizeof(int32_t), s));
    DMK_HIP(hipMemsetAsync(P->psi_slot, 0xff, nbox * sizeof(int32_t), s));
    if (P->nfout)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nfout)), dim3(TPB), 0, s, P->l_fout, P->nfout, P->proxy_slot);
    if (P->nanc)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nanc)), dim3(TPB), 0, s, P->l_anc, P->nanc, P->local_slot);
    P->anc_read = talloc<uint8_t>(P, std::max<int64_t>(P->nanc, 1));
    DMK_HIP(hipMemsetAsync(P->anc_read, 0, std::max<int64_t>(P->nanc, 1), s));
    if (P->nanc)
        hipLaunchKernelGGL(k_anchor_read, dim3(nblk(P->nanc)), dim3(TPB), 0, s, P->l_anc, P->nanc, P->blevel, P->parent,
                           P->anchor, P->local_slot, P->anc_read);
    if (P->nfin)
        hipLaunchKernelGGL(k_slots, dim3(nblk(P->nfin)), dim3(TPB), 0, s, P->l_fin, P->nfin, P->psi_slot);

    // sibling groups for the diagonal translation (the roots first, then the
    // parents level by level)
    {
        uint8_t *f_oct = S.get<uint8_t>(nbox);
        DMK_HIP(hipMemsetAsync(f_oct, 0, nbox, s));
        if (P->nfin)
            hipLaunchKernelGGL(k_oct_flag, dim3(nblk(P->nfin)), dim3(TPB), 0, s, P->l_fin, P->nfin, P->parent, f_oct);
        int32_t *octs = S.get<int32_t>(nbox + 1);
        int64_t m = select_indices(S, f_oct, 0, nbox, octs, s);
        // roots with F_in: the root's only colleague is itself
        const int np = P->nprob;
        std::vector<int32_t> rpsi(np), rphi(np);
        DMK_HIP(hipMemcpyAsync(rpsi.data(), P->psi_slot, np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipMemcpyAsync(rphi.data(), P->proxy_slot, np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> hd, hs, hl, hp;
        int root_cell = (D == 3) ? 21 : 5;  // cell (1,..,1)
        for (int b = 0; b < np; ++b) {
            if (rpsi[b] < 0) continue;
            for (int k = 0; k < NC; ++k) hd.push_back(k == 0 ? rpsi[b] : -1);
            for (int k = 0; k < NR; ++k) hs.push_back(k == root_cell ? rphi[b] : -1);
            hl.push_back(0);
            hp.push_back(b);
        }
        const int64_t r = (int64_t)hl.size();
        P->noct = m + r;
        P->oct_dst = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1) * NC);
        P->oct_src = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1) * NR);
        P->oct_level = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1));
        P->oct_prob = talloc<int32_t>(P, std::max<int64_t>(P->noct, 1));
        if (r) {
            DMK_HIP(hipMemcpyAsync(P->oct_dst, hd.data(), hd.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(P->oct_src, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(P->oct_level, hl.data(), hl.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipMemcpyAsync(P->oct_prob, hp.data(), hp.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            DMK_HIP(hipStreamSynchronize(s));
        }
        if (m)
            hipLaunchKernelGGL(k_oct_fill<D>, dim3((unsigned)m), dim3(64), 0, s, octs, m, P->child0, P->colleague,
                               P->bflags, P->blevel, P->bprob, P->proxy_slot, P->psi_slot, P->oct_dst + NC * r,
                               P->oct_src + NR * r, P->oct_level + r, P->oct_prob + r);
    }

    // targets grouped by the anchor of their leaf (leaf evaluation)
    {
        const int64_t nleaf = ll.leaf_off[L], nanc = ll.anc_off[L];
        P->anc_tbeg = talloc<int32_t>(P, nanc + 1);
        P->anc_tgt = talloc<int32_t>(P, std::max<int64_t>(P->n, 1));
        int32_t *cnt = S.get<int32_t>(nanc + 1);
        DMK_HIP(hipMemsetAsync(cnt, 0, (nanc + 1) * sizeof(int32_t), s));
        if (nleaf > 0) {
            int32_t *key = S.get<int32_t>(nleaf), *ident = S.get<int32_t>(nleaf);
            int32_t *skey = S.get<int32_t>(nleaf), *sleaf = S.get<int32_t>(nleaf);
            hipLaunchKernelGGL(k_leaf_keys, dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, P->anchor,
                               P->local_slot, P->tcount, key, ident, cnt);
            int kbits = 1;  // keys are anchor slots in [0, nanc)
            while ((int64_t(1) << kbits) < nanc) ++kbits;
            prim::sort_pairs(S, (const uint32_t *)key, (uint32_t *)skey, (const int32_t *)ident, sleaf, nleaf, kbits,
                             s);
            int32_t *lc = S.get<int32_t>(nleaf + 1), *pos = S.get<int32_t>(nleaf + 1);
            hipLaunchKernelGGL(k_leaf_counts, dim3(nblk(nleaf)), dim3(TPB), 0, s, sleaf, nleaf, P->tcount, lc);
            DMK_HIP(hipMemsetAsync(lc + nleaf, 0, sizeof(int32_t), s));
            prim::exclusive_scan(S, lc, pos, nleaf + 1, s);
            hipLaunchKernelGGL(k_fill_targets, dim3((unsigned)nleaf), dim3(TPB), 0, s, sleaf, nleaf, P->tstart,
                               P->tcount, pos, P->anc_tgt);
        }
        prim::exclusive_scan(S, cnt, P->anc_tbeg, nanc + 1, s);
    }

    // near lists over the leaf order
    const int64_t nleaf = P->nleaf;
    int32_t *lsd = S.get<int32_t>(L + 2);
    {
        std::vector<int32_t> h(L + 2);
        for (int l = 0; l <= L; ++l) h[l] = (int32_t)P->level_start[l];
        h[L + 1] = h[L];
        DMK_HIP(hipMemcpyAsync(lsd, h.data(), (L + 2) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    P->nl_off = talloc<int32_t>(P, nleaf + 1);
    if (nleaf > 0) {
        int32_t *cnt = S.get<int32_t>(nleaf);
        int64_t *pairs = S.get<int64_t>(nleaf);
        hipLaunchKernelGGL((k_near_lists<D, false>), dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, lsd, L, P->bkey,
                           P->blevel, P->parent, P->colleague, P->bflags, P->scount, P->tcount, cnt,
                           (const int32_t *)nullptr,
                           (int32_t *)nullptr, (int32_t *)nullptr, pairs);
        // exclusive sum over nleaf+1 entries needs a trailing zero in the input
        int32_t *cnt1 = S.get<int32_t>(nleaf + 1);
        DMK_HIP(hipMemcpyAsync(cnt1, cnt, nleaf * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        DMK_HIP(hipMemsetAsync(cnt1 + nleaf, 0, sizeof(int32_t), s));
        prim::exclusive_scan(S, cnt1, P->nl_off, nleaf + 1, s);
        int32_t total = 0;
        DMK_HIP(hipMemcpyAsync(&total, P->nl_off + nleaf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        {
            int32_t *mx = S.get<int32_t>(1);
            prim::reduce_max(cnt, nleaf, mx, s);
            int32_t hmx = 0;
            DMK_HIP(hipMemcpyAsync(&hmx, mx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DMK_HIP(hipStreamSynchronize(s));
            if (hmx > 1024)
                throw Error{DMK_ERR_UNSUPPORTED, "a leaf's residual list exceeds 1024 source boxes"};
            P->nl_max = hmx;
        }
        int64_t *psum = S.get<int64_t>(1);
        prim::reduce_sum(pairs, nleaf, psum, s);
        DMK_HIP(hipMemcpyAsync(&P->npairs, psum, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DMK_HIP(hipStreamSynchronize(s));
        P->nl_total = total;
        P->nl_src = talloc<int32_t>(P, total);
        P->nl_pre = talloc<int32_t>(P, total + nleaf);
        hipLaunchKernelGGL((k_near_lists<D, true>), dim3(nblk(nleaf)), dim3(TPB), 0, s, P->l_leaf, nleaf, lsd, L, P->bkey,
                           P->blevel, P->parent, P->colleague, P->bflags, P->scount, P->tcount, (int32_t *)nullptr,
                           (const int32_t *)P->nl_off, P->nl_src, P->nl_pre, (int64_t *)nullptr);
    } else {
        P->nl_src = talloc<int32_t>(P, 1);
        P->nl_pre = talloc<int32_t>(P, 1);
        DMK_HIP(hipMemsetAsync(P->nl_off, 0, sizeof(int32_t), s));
    }
    DMK_HIP(hipGetLastError());
    DMK_HIP(hipStreamSynchronize(s));
}

void build_lists(Plan *P, hipStream_t s)
{
    if (P->dim == 3) build_lists_t<3>(P, s);
    else build_lists_t<2>(P, s);
}

}  // namespace dmk
